// Fused single-pass bijective shuffle kernels for gfx950 (Algorithm 1, Sec. 4,
// in the fully fused form of Sec. 6's "Bijective2": one read and one write per
// kept item, no intermediate array in HBM).
//
// A workgroup of WAVES wavefronts owns a tile of 64*WAVES*ITEMS consecutive
// padded indices.  Wavefront w, lane l, item j handles index
//     tile*TILE + w*64*ITEMS + j*64 + l,
// so every item step of a wavefront covers 64 consecutive indices and one
// __ballot of the keep flags gives each lane its rank among them (mbcnt).
// Per tile:
//   1. cipher: ITEMS VariablePhilox evaluations per lane, interleaved for ILP;
//   2. keep = index < 2^k and f(index) < n; ballot -> wave-local ranks;
//   3. wave counts -> LDS -> tile total; wavefront 0 runs the decoupled
//      look-back for the tile's exclusive prefix;
//   4. the random gathers in[f(i)] and the stores at out[prefix + rank].
// Two schedules implement steps 3-4:
//   register  each lane keeps its own kept records in registers: the gathers
//             are issued right after the cipher (their latency overlaps the
//             scan) and every item step of a wavefront stores one contiguous
//             run (shuffle_single_kernel, shuffle_batched_kernel);
//   compacted the tile's kept images are first written to LDS in rank order,
//             then all lanes gather and store consecutive ranks, so memory
//             instructions run with full wavefronts; optionally the next
//             tile's cipher runs while the current tile's gathers are in
//             flight (shuffle_compact_kernel, shuffle_batched_compact_kernel).
// Tiles are handed out by atomic tickets in tile order, so a tile only ever
// waits on tiles already owned by running workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstddef>
#include <type_traits>

#include "kernels.h"

namespace bsd {

// ------------------------------------------------------------ payloads --
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int EB> struct Payload;
template <> struct Payload<0> { using T = uint32_t; };  // no payload (cipher + scan probe)
template <> struct Payload<1> { using T = uint8_t; };
template <> struct Payload<2> { using T = uint16_t; };
template <> struct Payload<4> { using T = uint32_t; };
template <> struct Payload<8> { using T = uint64_t; };
// 16-byte records: two 64-bit halves (an ext_vector of four words would be
// merged by the compiler with its neighbours in a register array into one
// wide vector value, which spills)
struct alignas(16) Rec16 { uint64_t lo, hi; };
template <> struct Payload<16> { using T = Rec16; };

template <int EB>
__device__ __forceinline__ typename Payload<EB>::T load_record(const uint8_t* __restrict__ base, uint64_t idx) {
  using T = typename Payload<EB>::T;
  if constexpr (EB == 16) {
    const u32x4 w = *reinterpret_cast<const u32x4*>(base + idx * 16u);
    return Rec16{uint64_t(w.x) | (uint64_t(w.y) << 32), uint64_t(w.z) | (uint64_t(w.w) << 32)};
  } else {
    return *reinterpret_cast<const T*>(base + idx * uint64_t(EB));
  }
}

template <int EB, bool NT>
__device__ __forceinline__ void store_record(uint8_t* __restrict__ base, uint64_t idx, typename Payload<EB>::T v) {
  if constexpr (EB == 16) {
    u32x4* p = reinterpret_cast<u32x4*>(base + idx * 16u);
    const u32x4 w = {uint32_t(v.lo), uint32_t(v.lo >> 32), uint32_t(v.hi), uint32_t(v.hi >> 32)};
    if constexpr (NT)
      __builtin_nontemporal_store(w, p);
    else
      *p = w;
  } else {
    using T = typename Payload<EB>::T;
    T* p = reinterpret_cast<T*>(base + idx * uint64_t(EB));
    if constexpr (NT)
      __builtin_nontemporal_store(v, p);
    else
      *p = v;
  }
}

// ------------------------------------------------------ workgroup state --
template <int WAVES>
struct TileLds {
  uint32_t ticket;
  uint32_t next_ticket;
  uint32_t cursor;  // XCD tickets: ranges this workgroup has found exhausted
  uint32_t xcd_first[kXcds + 1];  // XCD tickets: the ranges (fixed for the launch)
  uint32_t gen;
  uint32_t last;
  uint32_t limit;
  uint32_t wave_count[WAVES];
  uint64_t tile_exclusive;
};

// Tickets.  Single shuffles hand out tiles from one counter in launch order.
// Batched launches (XCD = true) may split the batch's tiles into kXcds ranges
// of whole segments (set up by the batch kernels before the launch); a
// workgroup takes tiles from the range of its own XCD first and moves on to
// the next XCD's range only when its own is exhausted, so a segment's tiles,
// and the random reads inside that segment, mostly stay in one L2.  Every
// range is handed out in tile order, so a tile still only waits on tiles
// owned by running workgroups.  Called by one lane at a time; lds.cursor
// counts the ranges that workgroup found exhausted.  Returns 0xFFFFFFFF when
// every range is exhausted.
template <bool XCD, int WAVES>
__device__ __forceinline__ uint32_t take_ticket(WorkspaceHeader* hdr, TileLds<WAVES>& lds) {
  if constexpr (!XCD) {
    return atomicAdd(&hdr->ticket, 1u);
  } else {
    const uint32_t home = blockIdx.x % kXcds;
    while (lds.cursor < kXcds) {
      const uint32_t x = (home + lds.cursor) % kXcds;
      const uint32_t begin = lds.xcd_first[x], end = lds.xcd_first[x + 1];
      if (begin < end) {
        const uint32_t t = begin + atomicAdd(&hdr->xcd_ticket[x], 1u);
        if (t < end) return t;
      }
      ++lds.cursor;
    }
    return 0xFFFFFFFFu;
  }
}

// The lane that takes a workgroup's tickets after the first one.  The register
// schedule with one tile in flight takes the next ticket once the current
// tile's prefix is known, and its latency overlaps the stores (a ticket taken
// earlier sits unstarted through the look-back wait while later tiles of its
// segment spin on it); with two tiles in flight, once every wave has counted
// its keeps; the compacted schedule takes it as the tile's compaction starts,
// which hides the atomic's latency behind the compaction.
template <int WAVES>
__device__ __forceinline__ bool ticket_lane() {
  constexpr uint32_t kTicketWave = WAVES > 1 ? 1u : 0u;
  return threadIdx.x == kTicketWave * 64u;
}

// Starts a workgroup: reads the launch generation (and the XCD ranges) and
// takes the first ticket.  Plain (relaxed) atomics: the header was last
// written by an earlier kernel, and kernel boundaries already make those
// writes visible; an acquire here would invalidate the XCD's L2 once per
// workgroup.
template <bool XCD = false, int WAVES>
__device__ __forceinline__ void group_begin(WorkspaceHeader* hdr, TileLds<WAVES>& lds) {
  if (threadIdx.x == 0) {
    lds.gen = __hip_atomic_load(&hdr->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lds.limit = __hip_atomic_load(&hdr->batch_tiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lds.cursor = 0;
    if constexpr (XCD) {
#pragma unroll
      for (uint32_t x = 0; x <= kXcds; ++x) lds.xcd_first[x] = hdr->xcd_first[x];
    }
    lds.ticket = take_ticket<XCD>(hdr, lds);
  }
  __syncthreads();
}

// Ends a workgroup.  The last one to finish resets the ticket and the done
// counter, raises the workspace's high-water mark of status words to this
// launch's `capacity`, and advances the generation; when the 24-bit tag wraps
// it first clears every status word up to that mark, so no stale word can
// carry a future tag.  Only status words are cleared: the batch tables that
// follow a batched launch's status words are not touched (the one-wavefront
// kernel that reads them runs before the tiled kernel, and a separate kernel
// zeroes them after it).
// Ordering without fences: a workgroup's last ticket fetch returned its value
// before the workgroup got here, and the wait below retires its status stores
// before it counts itself done; the done counter's modification order then
// puts every other workgroup's traffic before the last one's reset.
template <int WAVES>
__device__ __forceinline__ void group_end(WorkspaceHeader* hdr, uint64_t* status, uint32_t capacity,
                                          uint32_t gen, TileLds<WAVES>& lds) {
  __builtin_amdgcn_s_waitcnt(0);
  if (threadIdx.x == 0) {
    const uint32_t d = __hip_atomic_fetch_add(&hdr->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    lds.last = (d == gridDim.x - 1) ? 1u : 0u;
  }
  __syncthreads();
  if (lds.last) {
    const uint32_t next_gen = gen + 1;
    const uint32_t hwm = max(capacity, hdr->status_hwm);
    if ((next_gen & kTagMask) == 0) {
      for (uint32_t i = threadIdx.x; i < hwm; i += blockDim.x) atomic_store_agent(status + i, 0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    if (threadIdx.x < kXcds)
      __hip_atomic_store(&hdr->xcd_ticket[threadIdx.x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) {
      __hip_atomic_store(&hdr->status_hwm, hwm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&hdr->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&hdr->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&hdr->gen, next_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ------------------------------------------------------------- tile phases --
// A tile is processed in three phases so that a persistent workgroup can keep
// one tile's gathers in flight while it runs the next tile's cipher:
//   gather: cipher, keep flags, wave-local ranks, random loads issued;
//   scan:   workgroup scan of the wave counts and the decoupled look-back;
//   store:  kept records written at prefix + rank.
//
// MODE selects what a kept padded index i (image y = f(i), output rank r)
// produces:
//   kGather   out[r] = in[y]              the shuffle (Algorithm 1)
//   kIndices  out[r] = y                  the permutation itself (gather map)
//   kScatter  out[y] = in[r]              the inverse shuffle
//   kCount    nothing; tile totals only   first pass of the two-pass variant
// BIJ selects the bijection f:
//   kBijPhilox  VariablePhilox (Sec. 3.2), the shuffle's bijection
//   kBijTable   y read from a precomputed table of f over the padded domain
//               (the unfused variant's compaction pass)
//   kBijLcg     y = (a*i + c) mod 2^k, a odd (the LCG of Sec. 3.1)
enum Mode : int { kGather = 0, kIndices = 1, kScatter = 2, kCount = 3 };
enum Bijection : int { kBijPhilox = 0, kBijTable = 1, kBijLcg = 2 };

template <int EB, int MODE, bool WIDE>
struct ItemValue {
  using Idx = std::conditional_t<WIDE, uint64_t, uint32_t>;
  using T = std::conditional_t<MODE == kGather, typename Payload<EB>::T, Idx>;
};

template <int EB, int MODE, int ITEMS, bool WIDE>
struct PendingTile {
  typename ItemValue<EB, MODE, WIDE>::T val[ITEMS];  // gathered record, or the image y
  uint32_t keep_bits;                                // bit j: this lane keeps item j's index
  uint32_t wave_count;                               // kept indices of this wave (uniform)
};

template <int EB, int MODE, bool ODD, int WAVES, int ITEMS, bool WIDE, int BIJ = kBijPhilox,
          typename Keys = const uint32_t*>
__device__ __forceinline__ void tile_gather(PendingTile<EB, MODE, ITEMS, WIDE>& t, const uint8_t* __restrict__ in,
                                            uint64_t n, uint64_t domain, const CipherShape cs, uint32_t rounds,
                                            Keys keys, uint64_t tile_in_segment,
                                            const uint32_t* __restrict__ table = nullptr, uint64_t lcg_a = 0,
                                            uint64_t lcg_c = 0) {
  using Idx = std::conditional_t<WIDE, uint64_t, uint32_t>;
  constexpr uint32_t kTile = 64u * WAVES * ITEMS;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Idx tile_base = Idx(tile_in_segment) * Idx(kTile);
  const Idx base = tile_base + Idx(wave * (64u * ITEMS) + lane);
  // Tiles wholly inside the padded domain (every tile once 2^k >= tile size)
  // skip the per-index domain test.
  const bool whole_tile = uint64_t(tile_base) + kTile <= domain;

  // The cipher runs in sub-rounds of kSub items: the loads issued for one
  // sub-round are in flight while the next sub-round computes, and only kSub
  // cipher states are live at a time (register pressure sets occupancy).
  constexpr int kSub = ITEMS >= 16 ? 8 : ITEMS;
  const uint32_t wmask24 = cs.wmask & 0xFFFFFFu;
  const Idx x_last = Idx(domain - 1);
  const Idx y_last = Idx(n - 1);
  uint32_t wave_count = 0, keep_bits = 0;
#pragma unroll
  for (int s0 = 0; s0 < ITEMS; s0 += kSub) {
    // a sub-round wholly past the padded domain (small segments, the last
    // tile of a short shuffle) has nothing to keep: skip its cipher (the
    // test is uniform per wavefront, so this is a scalar branch)
    if (!whole_tile &&
        uint64_t(tile_base) + uint64_t(wave) * (64u * ITEMS) + uint64_t(s0) * 64u > uint64_t(x_last))
      continue;
    uint32_t L[kSub], R[kSub];
    uint32_t in_domain = whole_tile ? ~0u : 0u;  // bit j: index of item s0+j is < 2^k
    Idx x = base + Idx(s0 * 64);
#pragma unroll
    for (int j = 0; j < kSub; ++j, x += 64) {
      const bool inside = whole_tile || x <= x_last;
      if (!whole_tile) in_domain |= inside ? (1u << j) : 0u;
      if constexpr (BIJ == kBijTable) {
        L[j] = inside ? table[x] : 0u;  // the image itself (narrow domains only)
      } else if constexpr (BIJ == kBijPhilox) {
        L[j] = uint32_t(x >> cs.r) & wmask24;
        R[j] = uint32_t(x);
      }
    }
    if constexpr (BIJ == kBijPhilox) vp_encrypt<ODD, kSub>(L, R, cs, rounds, keys);
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
      Idx y;
      if constexpr (BIJ == kBijTable) {
        y = Idx(L[j]);
      } else if constexpr (BIJ == kBijLcg) {
        // arithmetic mod 2^32 (narrow) or 2^64 (wide), then mod 2^k
        y = (Idx(lcg_a) * (base + Idx((s0 + j) * 64)) + Idx(lcg_c)) & x_last;
      } else {
        y = (Idx(L[j]) << cs.r) | Idx(R[j] & cs.rmask);
      }
      // keep: the padded index is inside the domain and its image is < n
      // (as "<= last" so the narrow path compares in 32 bits: n, 2^k <= 2^32)
      const bool keep = ((in_domain >> j) & 1u) && (y <= y_last);
      const uint64_t m = __ballot(keep);
      keep_bits |= keep ? (1u << (s0 + j)) : 0u;
      if constexpr (MODE == kGather && EB > 0) {
        if (keep) t.val[s0 + j] = load_record<EB>(in, uint64_t(y));
      } else if constexpr (MODE == kIndices || MODE == kScatter) {
        t.val[s0 + j] = y;
      }
      wave_count += uint32_t(__builtin_popcountll(m));
    }
  }
  t.wave_count = wave_count;
  t.keep_bits = keep_bits;
}

// Returns this wave's output base: kept indices before the tile plus those
// of lower waves in the tile.  With LOOKBACK the tile's prefix comes from the
// decoupled look-back; otherwise from tile_prefix[status_idx] (written by an
// earlier pass).  Takes the workgroup's next ticket once every wave has
// counted its keeps; with LATE_TICKET only after the prefix is known (the
// caller then needs a barrier before it reads lds.next_ticket).
template <int WAVES, bool LOOKBACK = true, bool XCD = false, bool LATE_TICKET = false>
__device__ __forceinline__ uint64_t tile_scan(uint32_t wave_count, uint64_t* status, uint32_t status_first,
                                              uint32_t status_idx, uint32_t tag, WorkspaceHeader* hdr,
                                              TileLds<WAVES>& lds, Watchdog wd,
                                              const uint64_t* tile_prefix = nullptr) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (lane == 0) lds.wave_count[wave] = wave_count;
  __syncthreads();
  uint32_t wave_exclusive = 0, tile_total = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const uint32_t c = lds.wave_count[w];
    wave_exclusive += (uint32_t(w) < wave) ? c : 0u;
    tile_total += c;
  }
  if (!LATE_TICKET && ticket_lane<WAVES>()) lds.next_ticket = take_ticket<XCD>(hdr, lds);
  if (wave == 0) {
    uint64_t ex;
    if constexpr (LOOKBACK)
      ex = lookback_exclusive_prefix(status, status_first, status_idx, tag, uint64_t(tile_total), &hdr->error, wd);
    else
      ex = tile_prefix[status_idx];
    if (lane == 0) lds.tile_exclusive = ex;
  }
  __syncthreads();
  const uint64_t base = lds.tile_exclusive + wave_exclusive;
  if (LATE_TICKET && ticket_lane<WAVES>()) lds.next_ticket = take_ticket<XCD>(hdr, lds);
  return base;
}

// Writes the kept items: item j's kept lanes take consecutive ranks
// prefix + (kept before item j in this wave) + (kept lanes below this lane),
// the ballot and rank being recomputed here from the keep bits.  Ranks are
// < n by construction; the bound check only keeps a timed-out look-back from
// writing outside the buffer.  EB is the record size (kGather, kScatter) or
// the index size (kIndices: 4 or 8).
template <int EB, int MODE, int ITEMS, bool WIDE>
__device__ __forceinline__ void tile_store(const PendingTile<EB, MODE, ITEMS, WIDE>& t, const uint8_t* __restrict__ in,
                                           uint8_t* __restrict__ out, uint64_t n, uint64_t prefix,
                                           bool nontemporal) {
  if constexpr (MODE == kCount || EB == 0) {
    return;
  } else {
    uint64_t base = prefix;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const bool keep = (t.keep_bits >> j) & 1u;
      const uint64_t m = __ballot(keep);
      const uint32_t below =
          __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
      const uint64_t pos = base + below;
      if (keep && pos < n) {
        if constexpr (MODE == kGather) {
          if (nontemporal)
            store_record<EB, true>(out, pos, t.val[j]);
          else
            store_record<EB, false>(out, pos, t.val[j]);
        } else if constexpr (MODE == kIndices) {
          using IT = std::conditional_t<EB == 8, uint64_t, uint32_t>;
          reinterpret_cast<IT*>(out)[pos] = IT(t.val[j]);
        } else {  // kScatter: the record at rank pos goes back to position y
          store_record<EB, false>(out, uint64_t(t.val[j]), load_record<EB>(in, pos));
        }
      }
      base += uint64_t(__builtin_popcountll(m));
    }
  }
}

// -------------------------------------------------------- single kernel --
// Persistent loop over tickets.  DEPTH 2 keeps two tiles in flight: the
// gather phase of the next tile (cipher + loads issued) runs while the loads
// of the current tile are outstanding, then the current tile is stored.
// DEPTH 1 finishes each tile before starting the next (fewer registers).
// Minimum waves per SIMD the register budget is sized for (HIP's second
// launch-bounds argument).
template <int EB, int ITEMS, int DEPTH>
constexpr int kMinWavesPerSimd = (ITEMS <= 8 && DEPTH == 1 && EB <= 4) ? 8 : 1;

template <int EB, bool ODD, int WAVES, int ITEMS, int DEPTH, bool WIDE, int MODE = kGather, bool LOOKBACK = true,
          int BIJ = kBijPhilox>
__global__ __launch_bounds__(WAVES * 64, (kMinWavesPerSimd<EB, ITEMS, DEPTH>)) void shuffle_single_kernel(
    const SingleArgs a) {
  __shared__ TileLds<WAVES> lds;
  group_begin(a.hdr, lds);
  const uint32_t gen = lds.gen;
  const uint32_t tag = gen & kTagMask;
  const bool nt = a.nontemporal != 0;
  uint32_t tile = lds.ticket;
  if constexpr (DEPTH == 1) {
    PendingTile<EB, MODE, ITEMS, WIDE> cur;
    while (tile < a.num_tiles) {
      tile_gather<EB, MODE, ODD, WAVES, ITEMS, WIDE, BIJ>(cur, a.in, a.n, a.domain, a.cs, a.rounds, a.key, tile,
                                                          a.table, a.lcg_a, a.lcg_c);
      const uint64_t prefix =
          tile_scan<WAVES, LOOKBACK, false, true>(cur.wave_count, a.status, 0u, tile, tag, a.hdr, lds, a.wd,
                                                  a.tile_prefix);
      tile_store(cur, a.in, a.out, a.n, prefix, nt);
      __syncthreads();  // the next ticket, taken after the prefix, is in LDS
      tile = lds.next_ticket;
    }
  } else {
    PendingTile<EB, MODE, ITEMS, WIDE> cur, nxt;
    uint64_t cur_prefix = 0;
    if (tile < a.num_tiles) {
      tile_gather<EB, MODE, ODD, WAVES, ITEMS, WIDE, BIJ>(cur, a.in, a.n, a.domain, a.cs, a.rounds, a.key, tile,
                                                          a.table, a.lcg_a, a.lcg_c);
      cur_prefix = tile_scan<WAVES, LOOKBACK>(cur.wave_count, a.status, 0u, tile, tag, a.hdr, lds, a.wd,
                                              a.tile_prefix);
    }
    while (tile < a.num_tiles) {
      const uint32_t next = lds.next_ticket;
      const bool more = next < a.num_tiles;
      if (more)
        tile_gather<EB, MODE, ODD, WAVES, ITEMS, WIDE, BIJ>(nxt, a.in, a.n, a.domain, a.cs, a.rounds, a.key, next,
                                                            a.table, a.lcg_a, a.lcg_c);
      tile_store(cur, a.in, a.out, a.n, cur_prefix, nt);
      if (more) {
        cur_prefix = tile_scan<WAVES, LOOKBACK>(nxt.wave_count, a.status, 0u, next, tag, a.hdr, lds, a.wd,
                                                a.tile_prefix);
        cur = nxt;
      }
      tile = next;
    }
  }
  group_end(a.hdr, a.status, a.capacity, gen, lds);
}

// ------------------------------------------------ LDS-compacted tiles --
// Second tile schedule (32-bit images in LDS; WIDE: 64-bit images for domains
// above 2^32).  The register schedule above issues each item step's gathers
// and stores with only the kept lanes active: when about half the padded
// indices are rejected, twice as many half-empty memory instructions run as
// kept records need.  Here the kept images of a
// tile are first written to LDS in rank order; the workgroup's threads then
// gather and store consecutive ranks, so every memory instruction runs with
// all lanes active and each wavefront's stores cover 64 consecutive records.
// Per tile:
//   1. cipher and keep flags (ITEMS images per lane held in registers);
//   2. wave counts -> LDS -> wave offsets; kept images written to LDS at
//      their tile-local ranks; the next ticket is taken;
//   3. thread t gathers ranks t, t + T, t + 2T, ... (T threads) from in[];
//   4. wavefront 0 runs the look-back while those loads are in flight;
//   5. rank p is stored at out[prefix + p].
template <int WAVES, int ITEMS, bool WIDE = false>
struct CompactLds {
  TileLds<WAVES> t;
  std::conditional_t<WIDE, uint64_t, uint32_t> y[64 * WAVES * ITEMS];  // kept images of the tile, in rank order
};

// One tile as the compacted schedule sees it.
struct CompactView {
  const uint8_t* in;      // records of the tile's shuffle (segment)
  uint8_t* out;
  uint64_t n;             // records in the shuffle (bounds the stores)
  uint32_t status_first;  // status word of the shuffle's first tile
  uint32_t status_idx;    // the tile's own status word
};

// Compacts the tile whose images are in c into LDS, issues its gathers, finds
// its prefix and stores it.  The next ticket is taken as the call starts and
// published to the workgroup with the compaction.
// With PIPE, next_cipher(next) runs between the gathers and the stores so its
// VALU work covers the gathers' latency; it leaves the next tile's images in
// c.  Returns the next ticket.
template <int EB, int WAVES, int ITEMS, bool PIPE, bool LOOKBACK, bool XCD, bool WIDE, typename NextCipher>
__device__ __forceinline__ uint32_t compact_core(const CompactView& t, PendingTile<4, kIndices, ITEMS, WIDE>& c,
                                                 WorkspaceHeader* hdr, uint64_t* status,
                                                 const uint64_t* tile_prefix, uint32_t tag, bool nt,
                                                 CompactLds<WAVES, ITEMS, WIDE>& lds, Watchdog wd,
                                                 NextCipher&& next_cipher) {
  using T = typename Payload<EB>::T;
  constexpr uint32_t kThreads = 64u * WAVES;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t tk = ticket_lane<WAVES>() ? take_ticket<XCD>(hdr, lds.t) : 0u;
  if (lane == 0) lds.t.wave_count[wave] = c.wave_count;
  __syncthreads();
  uint32_t pos = 0, total = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    const uint32_t cnt = lds.t.wave_count[w];
    pos += (uint32_t(w) < wave) ? cnt : 0u;
    total += cnt;
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const bool keep = (c.keep_bits >> j) & 1u;
    const uint64_t m = __ballot(keep);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    if (keep) lds.y[pos + below] = c.val[j];
    pos += uint32_t(__builtin_popcountll(m));
  }
  if (ticket_lane<WAVES>()) lds.t.next_ticket = tk;
  __syncthreads();
  const uint32_t next = lds.t.next_ticket;
  // gathers for ranks threadIdx.x + q * kThreads, issued before the look-back;
  // lanes past the last rank re-read the last kept record (no per-lane branch,
  // so the payload registers stay independent values)
  // (EB == 0: no payload, the cipher, compaction and scan only)
  const uint32_t steps = (total + kThreads - 1) / kThreads;
  T v[ITEMS];
  if constexpr (EB > 0) {
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
      if (uint32_t(q) < steps) {
        const uint32_t p = min(threadIdx.x + uint32_t(q) * kThreads, total - 1);
        v[q] = load_record<EB>(t.in, lds.y[p]);
      }
    }
  }
  if (wave == 0) {
    uint64_t ex;
    if constexpr (LOOKBACK)
      ex = lookback_exclusive_prefix(status, t.status_first, t.status_idx, tag, uint64_t(total), &hdr->error, wd);
    else
      ex = tile_prefix[t.status_idx];  // written by an earlier scan pass
    if (lane == 0) lds.t.tile_exclusive = ex;
  }
  if constexpr (PIPE) next_cipher(next);
  __syncthreads();
  const uint64_t prefix = lds.t.tile_exclusive;
  if constexpr (EB > 0) {
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
      const uint32_t p = threadIdx.x + uint32_t(q) * kThreads;
      // ranks are < n by construction; the bound only keeps a timed-out
      // look-back from writing outside the buffer
      if (uint32_t(q) < steps && p < total && prefix + p < t.n) {
        if (nt)
          store_record<EB, true>(t.out, prefix + p, v[q]);
        else
          store_record<EB, false>(t.out, prefix + p, v[q]);
      }
    }
  }
  return next;
}

// Waves per SIMD the compacted kernel's register budget is sized for: with 8
// indices per lane and records of at most 4 bytes, two 16-wave workgroups fit
// on a CU (64 VGPRs), so one can compute while the other waits at a barrier or
// on the look-back.
template <int EB, int ITEMS, bool WIDE = false>
constexpr int kCompactMinWaves = (ITEMS <= 8 && EB <= 4 && !WIDE) ? 8 : 1;

// WIDE: domains above 2^32, 64-bit images in LDS.
template <int EB, bool ODD, int WAVES, int ITEMS, bool PIPE, int BIJ = kBijPhilox, bool LOOKBACK = true,
          bool WIDE = false>
__global__ __launch_bounds__(WAVES * 64, (kCompactMinWaves<EB, ITEMS, WIDE>)) void shuffle_compact_kernel(
    const SingleArgs a) {
  __shared__ CompactLds<WAVES, ITEMS, WIDE> lds;
  group_begin(a.hdr, lds.t);
  const uint32_t gen = lds.t.gen;
  const uint32_t tag = gen & kTagMask;
  const bool nt = a.nontemporal != 0;
  uint32_t tile = lds.t.ticket;
  PendingTile<4, kIndices, ITEMS, WIDE> c;
  auto cipher = [&](uint32_t t) {
    tile_gather<4, kIndices, ODD, WAVES, ITEMS, WIDE, BIJ>(c, nullptr, a.n, a.domain, a.cs, a.rounds, a.key, t,
                                                          a.table, a.lcg_a, a.lcg_c);
  };
  if (PIPE && tile < a.num_tiles) cipher(tile);
  while (tile < a.num_tiles) {
    if (!PIPE) cipher(tile);
    const CompactView v{a.in, a.out, a.n, 0u, tile};
    auto next_cipher = [&](uint32_t nx) {
      if (nx < a.num_tiles) cipher(nx);
    };
    tile = compact_core<EB, WAVES, ITEMS, PIPE, LOOKBACK, false, WIDE>(v, c, a.hdr, a.status, a.tile_prefix, tag,
                                                                       nt, lds, a.wd, next_cipher);
  }
  group_end(a.hdr, a.status, a.capacity, gen, lds.t);
}

// First pass of the two-pass scan variant: the kept count of every tile,
// written to tile_counts[tile] (no look-back, no payload).  One workgroup per
// tile, in any order.
template <bool ODD, int WAVES, int ITEMS>
__global__ __launch_bounds__(WAVES * 64) void tile_count_kernel(const SingleArgs a) {
  __shared__ uint32_t wave_counts[WAVES];
  for (uint32_t tile = blockIdx.x; tile < a.num_tiles; tile += gridDim.x) {
    PendingTile<0, kCount, ITEMS, false> t;
    tile_gather<0, kCount, ODD, WAVES, ITEMS, false>(t, nullptr, a.n, a.domain, a.cs, a.rounds, a.key, tile);
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) wave_counts[wave] = t.wave_count;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t total = 0;
      for (int w = 0; w < WAVES; ++w) total += wave_counts[w];
      a.tile_counts[tile] = total;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- batched kernels --
__device__ __forceinline__ uint64_t splitmix64_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t domain_bits_dev(uint64_t n) {
  uint32_t k = (n <= 1) ? 0u : 64u - uint32_t(__builtin_clzll(n - 1));
  return k < 4u ? 4u : k;
}

// Uniform view of one tile of a batch: its segment's slice and cipher.
struct BatchTile {
  const uint8_t* in;
  uint8_t* out;
  uint64_t n;
  uint64_t domain;
  ConstKeys keys;  // the segment's masked round keys (batch table in the workspace)
  CipherShape cs;
  uint32_t first_tile;
  uint32_t tile_in_segment;
  bool odd;
};

// The batch tables (tile -> segment, segment records, keys) are written by
// the preparation kernels and only read here, so they are read through the
// constant address space: with a uniform tile index these are scalar loads.
using ConstSegments = const __attribute__((address_space(4))) SegmentInfo*;

template <int EB>
__device__ __forceinline__ BatchTile batch_tile(const BatchArgs& a, uint32_t tile) {
  BatchTile b;
  tile = __builtin_amdgcn_readfirstlane(tile);
  const uint32_t s = __builtin_amdgcn_readfirstlane(global_keys(a.tile_segment)[tile]);
  const ConstSegments seg = (ConstSegments)a.segs + s;
  const uint64_t first = seg->first;
  const uint32_t first_tile = seg->first_tile;
  const uint32_t k = __builtin_amdgcn_readfirstlane(seg->k);
  b.cs.w = k >> 1;
  b.cs.r = k - b.cs.w;
  b.cs.wmask = (1u << b.cs.w) - 1u;
  b.cs.rmask = (1u << b.cs.r) - 1u;
  b.keys = global_keys(a.keys + uint64_t(s) * (a.rounds + 1));
  b.in = a.in + first * uint64_t(EB);
  b.out = a.out + first * uint64_t(EB);
  b.n = seg->n;
  b.domain = uint64_t(1) << k;
  b.first_tile = first_tile;
  b.tile_in_segment = tile - first_tile;
  b.odd = (k & 1u) != 0;
  return b;
}

template <int EB, int WAVES, int ITEMS>
__device__ __forceinline__ void batch_gather(PendingTile<EB, kGather, ITEMS, false>& t, const BatchTile& b,
                                             uint32_t rounds) {
  if (b.odd)
    tile_gather<EB, kGather, true, WAVES, ITEMS, false>(t, b.in, b.n, b.domain, b.cs, rounds, b.keys,
                                                        b.tile_in_segment);
  else
    tile_gather<EB, kGather, false, WAVES, ITEMS, false>(t, b.in, b.n, b.domain, b.cs, rounds, b.keys,
                                                         b.tile_in_segment);
}

template <int EB, int WAVES, int ITEMS, int DEPTH>
__global__ __launch_bounds__(WAVES * 64, (kMinWavesPerSimd<EB, ITEMS, DEPTH>)) void shuffle_batched_kernel(
    const BatchArgs a) {
  __shared__ TileLds<WAVES> lds;
  group_begin<true>(a.hdr, lds);
  const uint32_t gen = lds.gen;
  const uint32_t tag = gen & kTagMask;
  const uint32_t limit = lds.limit;
  const bool nt = a.nontemporal != 0;
  uint32_t tile = lds.ticket;
  if constexpr (DEPTH == 1) {
    PendingTile<EB, kGather, ITEMS, false> cur;
    while (tile < limit) {
      const BatchTile b = batch_tile<EB>(a, tile);
      batch_gather<EB, WAVES, ITEMS>(cur, b, a.rounds);
      const uint64_t prefix =
          tile_scan<WAVES, true, true, true>(cur.wave_count, a.status, b.first_tile, tile, tag, a.hdr, lds, a.wd);
      tile_store(cur, nullptr, b.out, b.n, prefix, nt);
      __syncthreads();  // the next ticket, taken after the prefix, is in LDS
      tile = lds.next_ticket;
    }
  } else {
    PendingTile<EB, kGather, ITEMS, false> cur, nxt;
    uint64_t cur_prefix = 0;
    uint8_t* cur_out = nullptr;
    uint64_t cur_n = 0;
    if (tile < limit) {
      const BatchTile b = batch_tile<EB>(a, tile);
      batch_gather<EB, WAVES, ITEMS>(cur, b, a.rounds);
      cur_prefix =
          tile_scan<WAVES, true, true>(cur.wave_count, a.status, b.first_tile, tile, tag, a.hdr, lds, a.wd);
      cur_out = b.out;
      cur_n = b.n;
    }
    while (tile < limit) {
      const uint32_t next = lds.next_ticket;
      const bool more = next < limit;
      BatchTile b;
      if (more) {
        b = batch_tile<EB>(a, next);
        batch_gather<EB, WAVES, ITEMS>(nxt, b, a.rounds);
      }
      tile_store(cur, nullptr, cur_out, cur_n, cur_prefix, nt);
      if (more) {
        cur_prefix =
            tile_scan<WAVES, true, true>(nxt.wave_count, a.status, b.first_tile, next, tag, a.hdr, lds, a.wd);
        cur = nxt;
        cur_out = b.out;
        cur_n = b.n;
      }
      tile = next;
    }
  }
  group_end(a.hdr, a.status, a.capacity, gen, lds);
}

// Batched form of the compacted schedule: a tile's segment (slice, domain,
// keys, first status word) is looked up per tile; with PIPE the next tile's
// segment and cipher are taken while the current tile's gathers are in flight.
// (The pipelined batched form keeps the next tile's segment record live as
// well; it does not fit in 64 VGPRs, so it is sized for one workgroup per CU.)
template <int EB, int ITEMS, bool PIPE>
constexpr int kBatchCompactMinWaves = PIPE ? 1 : kCompactMinWaves<EB, ITEMS>;

template <int EB, int WAVES, int ITEMS, bool PIPE>
__global__ __launch_bounds__(WAVES * 64, (kBatchCompactMinWaves<EB, ITEMS, PIPE>)) void shuffle_batched_compact_kernel(
    const BatchArgs a) {
  __shared__ CompactLds<WAVES, ITEMS> lds;
  group_begin<true>(a.hdr, lds.t);
  const uint32_t gen = lds.t.gen;
  const uint32_t tag = gen & kTagMask;
  const uint32_t limit = lds.t.limit;
  const bool nt = a.nontemporal != 0;
  uint32_t tile = lds.t.ticket;
  PendingTile<4, kIndices, ITEMS, false> c;
  auto cipher = [&](const BatchTile& b) {
    if (b.odd)
      tile_gather<4, kIndices, true, WAVES, ITEMS, false>(c, nullptr, b.n, b.domain, b.cs, a.rounds, b.keys,
                                                          b.tile_in_segment);
    else
      tile_gather<4, kIndices, false, WAVES, ITEMS, false>(c, nullptr, b.n, b.domain, b.cs, a.rounds, b.keys,
                                                           b.tile_in_segment);
  };
  BatchTile b;
  if (PIPE && tile < limit) {
    b = batch_tile<EB>(a, tile);
    cipher(b);
  }
  while (tile < limit) {
    if (!PIPE) {
      b = batch_tile<EB>(a, tile);
      cipher(b);
    }
    const CompactView v{b.in, b.out, b.n, b.first_tile, tile};
    BatchTile nb;
    auto next_cipher = [&](uint32_t nx) {
      if (nx < limit) {
        nb = batch_tile<EB>(a, nx);
        cipher(nb);
      }
    };
    tile = compact_core<EB, WAVES, ITEMS, PIPE, true, true, false>(v, c, a.hdr, a.status, nullptr, tag, nt, lds,
                                                                   a.wd, next_cipher);
    if (PIPE) b = nb;
  }
  group_end(a.hdr, a.status, a.capacity, gen, lds.t);
}

// Variants outside the main shape table use one fixed shape.
constexpr int kAltWaves = 16, kAltItems = 16;

template <int EB, int MODE, bool LOOKBACK, int BIJ>
SingleFn pick_variant_eb(bool odd, bool wide) {
  if constexpr (BIJ == kBijTable) {  // the table holds 32-bit images: narrow domains only
    if (wide) return nullptr;
    return odd ? &shuffle_single_kernel<EB, true, kAltWaves, kAltItems, 1, false, MODE, LOOKBACK, BIJ>
               : &shuffle_single_kernel<EB, false, kAltWaves, kAltItems, 1, false, MODE, LOOKBACK, BIJ>;
  } else if constexpr (BIJ == kBijLcg) {  // no Feistel halves: odd and even k share a kernel
    if (wide) return &shuffle_single_kernel<EB, false, kWideWaves, kWideItems, 1, true, MODE, LOOKBACK, BIJ>;
    return &shuffle_compact_kernel<EB, false, kAltWaves, kAltItems, true, BIJ, LOOKBACK>;
  } else {
    if (wide) {
      if constexpr (!LOOKBACK) return nullptr;
      if constexpr (MODE == kIndices && EB == 4) return nullptr;  // 64-bit images need 8-byte indices
      return odd ? &shuffle_single_kernel<EB, true, kWideWaves, kWideItems, 1, true, MODE, LOOKBACK, BIJ>
                 : &shuffle_single_kernel<EB, false, kWideWaves, kWideItems, 1, true, MODE, LOOKBACK, BIJ>;
    }
    if constexpr (MODE == kGather)  // the two-pass form: same tile schedule as the fused kernel
      return odd ? &shuffle_compact_kernel<EB, true, kAltWaves, kAltItems, true, BIJ, LOOKBACK>
                 : &shuffle_compact_kernel<EB, false, kAltWaves, kAltItems, true, BIJ, LOOKBACK>;
    return odd ? &shuffle_single_kernel<EB, true, kAltWaves, kAltItems, 1, false, MODE, LOOKBACK, BIJ>
               : &shuffle_single_kernel<EB, false, kAltWaves, kAltItems, 1, false, MODE, LOOKBACK, BIJ>;
  }
}

// ------------------------------------------------------------ dispatch --
// Kernels are instantiated per element size in separate translation units
// (inst_eb*.hip) so the build compiles them in parallel.  Supported shapes
// (waves, items, depth) are listed once in BSD_FOR_EACH_SHAPE (kernels.h).
template <int EB, bool ODD, bool WIDE>
SingleFn pick_single_shape(const LaunchConfig& c) {
  if constexpr (WIDE) {  // one shape: compacted, pipelined, 64-bit images
    return &shuffle_compact_kernel<EB, ODD, kWideWaves, kWideItems, true, kBijPhilox, true, true>;
  } else {
    if (c.depth == kDepthCompact || c.depth == kDepthCompactPipe) {
      const bool pipe = c.depth == kDepthCompactPipe;
#define BSD_PICK(W, I)                  \
  if (c.waves == W && c.items == I)     \
    return pipe ? &shuffle_compact_kernel<EB, ODD, W, I, true> : &shuffle_compact_kernel<EB, ODD, W, I, false>;
      BSD_FOR_EACH_COMPACT_SHAPE(BSD_PICK)
#undef BSD_PICK
      return nullptr;
    }
#define BSD_PICK(W, I, D) \
  if (c.waves == W && c.items == I && c.depth == D) return &shuffle_single_kernel<EB, ODD, W, I, D, false>;
    BSD_FOR_EACH_SHAPE(BSD_PICK)
#undef BSD_PICK
    return nullptr;
  }
}

template <int EB>
SingleFn pick_single_eb(bool odd, bool wide, const LaunchConfig& c) {
  if (wide) return odd ? pick_single_shape<EB, true, true>(c) : pick_single_shape<EB, false, true>(c);
  return odd ? pick_single_shape<EB, true, false>(c) : pick_single_shape<EB, false, false>(c);
}

// Segments whose padded domain is at most 64 x kSmallSegmentItems indices:
// one wavefront shuffles a whole segment with its items in registers, ranks
// from the wavefront's ballots alone (Algorithm 1's scan within one
// wavefront), so there is no tile, no LDS, no barrier and no look-back; a
// segment costs a few microseconds of latency instead of a workgroup's tile.
// Workgroups of one wavefront take segments in a fixed stride (no tickets:
// nothing waits on anything).  A batch the preparation kernel rejected is
// left untouched.
template <int EB>
__global__ __launch_bounds__(64) void shuffle_batched_small_kernel(const BatchArgs a) {
  if (__hip_atomic_load(&a.hdr->batch_bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const bool nt = a.nontemporal != 0;
  for (uint32_t s = blockIdx.x; s < a.num_segments; s += gridDim.x) {
    const ConstSegments seg = (ConstSegments)a.segs + s;
    const uint64_t n = seg->n;
    const uint32_t k = __builtin_amdgcn_readfirstlane(seg->k);
    if (n == 0 || k > a.small_bits) continue;
    const uint64_t first = seg->first;
    CipherShape cs;
    cs.w = k >> 1;
    cs.r = k - cs.w;
    cs.wmask = (1u << cs.w) - 1u;
    cs.rmask = (1u << cs.r) - 1u;
    const ConstKeys keys = global_keys(a.keys + uint64_t(s) * (a.rounds + 1));
    const uint8_t* in = a.in + first * uint64_t(EB);
    uint8_t* out = a.out + first * uint64_t(EB);
    PendingTile<EB, kGather, kSmallSegmentItems, false> t;
    if (k & 1u)
      tile_gather<EB, kGather, true, 1, kSmallSegmentItems, false>(t, in, n, uint64_t(1) << k, cs, a.rounds, keys, 0);
    else
      tile_gather<EB, kGather, false, 1, kSmallSegmentItems, false>(t, in, n, uint64_t(1) << k, cs, a.rounds, keys,
                                                                    0);
    tile_store(t, nullptr, out, n, 0, nt);
  }
}

template <int EB>
BatchFn pick_batch_small_eb() {
  return &shuffle_batched_small_kernel<EB>;
}

template <int EB>
BatchFn pick_batch_eb(const LaunchConfig& c) {
  if (c.depth == kDepthCompact || c.depth == kDepthCompactPipe) {
    const bool pipe = c.depth == kDepthCompactPipe;
#define BSD_PICK(W, I)              \
  if (c.waves == W && c.items == I) \
    return pipe ? &shuffle_batched_compact_kernel<EB, W, I, true> : &shuffle_batched_compact_kernel<EB, W, I, false>;
    BSD_FOR_EACH_COMPACT_SHAPE(BSD_PICK)
#undef BSD_PICK
    return nullptr;
  }
#define BSD_PICK(W, I, D) \
  if (c.waves == W && c.items == I && c.depth == D) return &shuffle_batched_kernel<EB, W, I, D>;
  BSD_FOR_EACH_SHAPE(BSD_PICK)
#undef BSD_PICK
  return nullptr;
}

}  // namespace bsd
