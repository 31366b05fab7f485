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

// One round.  R arrives with this round's key already xored into it
// (Rk = R ^ key_r) and leaves with the next round's key xored in, so the key
// never costs an instruction on the L path and R' is a fresh register (the
// 64-bit product's halves are not carried across rounds).  Keys must be
// masked to the half width, so bit w of Rk is still the extra bit b; the key
// after the last round is 0, which leaves the plain R.  L < 2^24 is required;
// callers pass wmask & 0xFFFFFF so the compiler can see it.
template <bool ODD>
__device__ __forceinline__ void vp_round(uint32_t& L, uint32_t& Rk, uint32_t key_next, uint32_t w,
                                         uint32_t wmask24) {
  const uint64_t p = uint64_t(kM0Lo) * uint64_t(L);  // v_mad_u64_u32
  const uint32_t lo = uint32_t(p);
  // hi = (M0hi mod 2^24) * L + high word of M0lo * L.  Written as one
  // v_mad_u32_u24: left to itself the compiler widens this into a second
  // 64-bit multiply-add plus register-pair copies.
  uint32_t hi;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(hi) : "s"(kM0Hi24), "v"(L), "v"(uint32_t(p >> 32)));
  const uint32_t Ln = (hi ^ Rk) & wmask24;  // F(L) xor R (key already in Rk)
  uint32_t Rn;
  if constexpr (ODD) {
    Rn = ((lo << 1) | __builtin_amdgcn_ubfe(Rk, w, 1u)) ^ key_next;
  } else {
    Rn = lo ^ key_next;
  }
  L = Ln;
  Rk = Rn;
}

// 32-bit words in global memory that nothing writes while the reading kernel
// runs (the batch tables: round keys, tile -> segment), seen through the
// constant address space: uniform loads of them then compile to scalar loads
// even in kernels that also store to global memory (through a generic pointer
// the round keys cost one vector load per round and wavefront).  Only for
// pointers into global memory.
using ConstKeys = const __attribute__((address_space(4))) uint32_t*;
__device__ __forceinline__ ConstKeys global_keys(const uint32_t* p) { return (ConstKeys)p; }

// Encrypts ITEMS independent blocks, interleaved round by round so that the
// ITEMS dependency chains fill the VALU pipeline.  keys[0..rounds] are the
// round keys masked to the half width followed by a 0; they are read one per
// round from uniform memory (scalar loads: kernel arguments, or ConstKeys),
// which keeps them out of the scalar register file.
template <bool ODD, int ITEMS, typename Keys>
__device__ __forceinline__ void vp_encrypt(uint32_t (&L)[ITEMS], uint32_t (&R)[ITEMS], const CipherShape& cs,
                                           uint32_t rounds, Keys keys) {
  const uint32_t wmask24 = cs.wmask & 0xFFFFFFu;
  const uint32_t key0 = keys[0];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) R[j] ^= key0;
  for (uint32_t rr = 0; rr < rounds; ++rr) {
    const uint32_t key_next = keys[rr + 1];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) vp_round<ODD>(L[j], R[j], key_next, cs.w, wmask24);
  }
}

// The inverse, by the three steps of Sec. 3.2 applied to one round's output
// (L', R') in the same layout (for odd k bit w of R is the extra bit):
//   B      = bits [1, w] of R' (odd k; bit 0 is the old extra bit) or R'
//   L      = B^-1(B) = M0^-1 * B mod 2^w
//   R      = F(L) ^ L' on bits [0, w), the old extra bit back in bit w
// Only the low w <= 24 bits of M0^-1 * B survive, so one 24-bit multiply
// (v_mul_u32_u24) with M0^-1 mod 2^24 gives L; F(L) reuses the forward
// round's product.  Keys are masked to the half width.
//
// Bits of R above r (above w for even k) may hold leftovers between rounds:
// they only reach bits at or above w of the next product M0^-1 * B, which the
// mask on L drops.  So R is never masked inside the loop, only once at the end
// of vp_decrypt, and an even-k round is five VALU instructions (24-bit
// multiply, mask, 32x32 high product, 24-bit multiply-add, three-input xor);
// odd k adds the shift that extracts B and the two that move the extra bit.
// The 24-bit multiply is written out: the compiler otherwise proves that a
// full 32-bit multiply gives the same masked bits and emits v_mul_lo_u32.
constexpr uint64_t kM0Inverse = 0xF5F365BD212BDF9Bull;
static_assert(kM0 * kM0Inverse == 1, "kM0Inverse is the inverse of M0 mod 2^64");
constexpr uint32_t kM0InvLo24 = static_cast<uint32_t>(kM0Inverse) & 0xFFFFFFu;

template <bool ODD>
__device__ __forceinline__ void vp_round_inverse(uint32_t& L, uint32_t& R, uint32_t key, uint32_t w,
                                                 uint32_t wmask24) {
  const uint32_t B = ODD ? (R >> 1) : R;
  uint32_t t;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(t) : "s"(kM0InvLo24), "v"(B));
  const uint32_t Lp = t & wmask24;
  const uint64_t p = uint64_t(kM0Lo) * uint64_t(Lp);
  uint32_t hi;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(hi) : "s"(kM0Hi24), "v"(Lp), "v"(uint32_t(p >> 32)));
  // low = hi ^ L ^ key as one v_bitop3_b32 (truth table 0x96; the compiler
  // emits two xors): bits [0, w) are R's, above them leftovers
  uint32_t low;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(low) : "v"(hi), "v"(L), "s"(key));
  if constexpr (ODD) {
    // bits [0, w) from low, the extra bit (bit 0 of R') into bit w: one
    // shift and one bitfield insert (v_bfi_b32: mask ? low : R << w)
    const uint32_t Rs = R << w;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(R) : "s"(wmask24), "v"(low), "v"(Rs));
  } else {
    R = low;
  }
  L = Lp;
}

// Decrypts ITEMS independent blocks (L < 2^w, R < 2^r), rounds in reverse,
// interleaved like vp_encrypt.  keys[0..rounds) are masked to the half width.
// Two rounds per loop step (an odd round count takes its last round first):
// with one round per step every state register is rewritten while its old
// value is still live, which costs a register copy per block and round.
// Leaves L < 2^w and R < 2^r.
template <bool ODD, int ITEMS>
__device__ __forceinline__ void vp_decrypt(uint32_t (&L)[ITEMS], uint32_t (&R)[ITEMS], const CipherShape& cs,
                                           uint32_t rounds, const uint32_t* __restrict__ keys) {
  const uint32_t wmask24 = cs.wmask & 0xFFFFFFu;
  uint32_t rr = rounds;
  if (rr & 1u) {
    --rr;
    const uint32_t key = keys[rr];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) vp_round_inverse<ODD>(L[j], R[j], key, cs.w, wmask24);
  }
  for (; rr != 0; rr -= 2) {
    const uint32_t k1 = keys[rr - 1], k0 = keys[rr - 2];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) vp_round_inverse<ODD>(L[j], R[j], k1, cs.w, wmask24);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) vp_round_inverse<ODD>(L[j], R[j], k0, cs.w, wmask24);
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) R[j] &= cs.rmask;
}

}  // namespace bsd
