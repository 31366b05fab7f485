// VariablePhilox round on gfx950 (device code).
//
// The cipher of Sec. 3.2 on k-bit blocks, k = w + r with w = floor(k/2)
// (left half) and r = ceil(k/2) (right part; when k is odd its top bit is the
// extra bit b of the paper's construction).  The state is held as two 32-bit
// registers: L (w bits) and R (the low r bits matter; bits above may hold
// leftovers, every consumer masks or extracts what it needs).  One round:
//
//   (hi, lo) = words of the 64-bit product M0 * L
//   L'       = (hi ^ key ^ R) & wmask                  F(L) xor R
//   R'       = lo                  (k even)            B(L)
//   R'       = (lo << 1) | bit_w(R) (k odd)            G(B(L), b): b enters
//                                                      below B(L); the top
//                                                      bit moves into bit w
//
// Only bits [0, w) of lo and bits [32, 32 + w) of M0 * L ever survive, and
// w <= 24 (k <= 49), so
//     M0 * L = M0lo * L + 2^32 * (M0hi * L)
// needs one 32x32->64 product (v_mad_u64_u32, full rate on gfx950) and one
// 24-bit multiply-add for the low bits of M0hi * L (v_mad_u32_u24).  With the
// xor and a masked three-input xor (v_bitop3_b32) an even-k round is four
// VALU instructions; odd k adds a bit extract and a shift-or.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsd {

// Philox's 64-bit multiplier, the constant VariablePhilox uses (Sec. 3.2).
constexpr uint64_t kM0 = 0xD2B74407B1CE6E93ull;
constexpr uint32_t kM0Lo = static_cast<uint32_t>(kM0);
constexpr uint32_t kM0Hi24 = static_cast<uint32_t>(kM0 >> 32) & 0xFFFFFFu;

// Uniform description of one cipher domain [0, 2^k).
struct CipherShape {
  uint32_t w;      // left width, floor(k/2)
  uint32_t r;      // right width, k - w
  uint32_t wmask;  // 2^w - 1
  uint32_t rmask;  // 2^r - 1
};

// L < 2^24 is required; callers pass wmask & 0xFFFFFF so the compiler can see
// it and select the 24-bit multiply.
template <bool ODD>
__device__ __forceinline__ void vp_round(uint32_t& L, uint32_t& R, uint32_t key, uint32_t w, uint32_t wmask24) {
  const uint64_t p = uint64_t(kM0Lo) * uint64_t(L);
  const uint32_t lo = uint32_t(p);
  const uint32_t hi = uint32_t(p >> 32) + kM0Hi24 * L;
  const uint32_t Ln = (hi ^ key ^ R) & wmask24;
  uint32_t Rn;
  if constexpr (ODD) {
    Rn = (lo << 1) | __builtin_amdgcn_ubfe(R, w, 1u);
  } else {
    Rn = lo;
  }
  L = Ln;
  R = Rn;
}

// Encrypts ITEMS independent blocks, interleaved round by round so that the
// ITEMS dependency chains fill the VALU pipeline.  Round keys are read one
// per round from uniform memory (scalar loads), which keeps them out of the
// scalar register file.
template <bool ODD, int ITEMS>
__device__ __forceinline__ void vp_encrypt(uint32_t (&L)[ITEMS], uint32_t (&R)[ITEMS], const CipherShape& cs,
                                           uint32_t rounds, const uint32_t* __restrict__ keys) {
  const uint32_t wmask24 = cs.wmask & 0xFFFFFFu;
  for (uint32_t rr = 0; rr < rounds; ++rr) {
    const uint32_t key = keys[rr];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) vp_round<ODD>(L[j], R[j], key, cs.w, wmask24);
  }
}

}  // namespace bsd
