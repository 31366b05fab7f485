// The keyed bijection on its own (bs_bijection): f, or its inverse, applied
// elementwise to 64-bit values.
//
// Both directions are the shuffle's own device code: vp_encrypt (the round
// the shuffle kernels run) and vp_decrypt (Sec. 3.2's inversion, also used by
// the f^-1 form of the un-shuffle).  Not a hot path: one element per lane, a
// grid-stride loop.
#include "kernels.h"

namespace bsd {
namespace {

constexpr int kBlock = 256;

template <bool ODD>
__device__ __forceinline__ uint64_t apply_forward(uint64_t x, const BijectionArgs& a) {
  uint32_t L[1] = {uint32_t(x >> a.cs.r) & a.cs.wmask};
  uint32_t R[1] = {uint32_t(x) & a.cs.rmask};
  vp_encrypt<ODD, 1>(L, R, a.cs, a.rounds, a.key);
  return (uint64_t(L[0]) << a.cs.r) | (R[0] & a.cs.rmask);
}

template <bool ODD>
__device__ __forceinline__ uint64_t apply_inverse(uint64_t y, const BijectionArgs& a) {
  uint32_t L[1] = {uint32_t(y >> a.cs.r) & a.cs.wmask};
  uint32_t R[1] = {uint32_t(y) & a.cs.rmask};
  vp_decrypt<ODD, 1>(L, R, a.cs, a.rounds, a.key);
  return (uint64_t(L[0]) << a.cs.r) | R[0];
}

template <bool ODD, bool INVERSE>
__global__ __launch_bounds__(kBlock) void bijection_kernel(const BijectionArgs a) {
  const uint64_t domain_mask = (uint64_t(1) << (a.cs.w + a.cs.r)) - 1;
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < a.count; i += stride) {
    const uint64_t v = a.in[i] & domain_mask;
    a.out[i] = INVERSE ? apply_inverse<ODD>(v, a) : apply_forward<ODD>(v, a);
  }
}

}  // namespace

hipError_t launch_bijection(const BijectionArgs& a, hipStream_t stream) {
  const uint64_t want = (a.count + kBlock - 1) / kBlock;
  const dim3 grid(uint32_t(want < 65536 ? want : 65536));
  const bool odd = (a.cs.w + a.cs.r) & 1u;
  if (odd && a.inverse)
    hipLaunchKernelGGL((bijection_kernel<true, true>), grid, dim3(kBlock), 0, stream, a);
  else if (odd)
    hipLaunchKernelGGL((bijection_kernel<true, false>), grid, dim3(kBlock), 0, stream, a);
  else if (a.inverse)
    hipLaunchKernelGGL((bijection_kernel<false, true>), grid, dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL((bijection_kernel<false, false>), grid, dim3(kBlock), 0, stream, a);
  return hipGetLastError();
}

}  // namespace bsd
