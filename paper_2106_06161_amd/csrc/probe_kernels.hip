// Measurement kernels: the device-copy and random-gather ceilings the
// shuffle is reported against (the paper's yardstick for any GPU shuffle is
// a random gather, Sec. 2.2 and Sec. 6).  Declared in include/bshuffle_probe.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bshuffle_probe.h"

namespace {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Each lane moves kCopyUnroll 16-byte vectors per step, all loads issued
// before the stores, so every wavefront keeps several reads in flight.
constexpr int kCopyUnroll = 4;
__global__ __launch_bounds__(256) void copy16_kernel(const u32x4* __restrict__ in, u32x4* __restrict__ out,
                                                     uint64_t vecs) {
  const uint64_t step = uint64_t(gridDim.x) * 256 * kCopyUnroll;
  for (uint64_t base = uint64_t(blockIdx.x) * 256 * kCopyUnroll + threadIdx.x; base < vecs; base += step) {
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int j = 0; j < kCopyUnroll; ++j) {
      const uint64_t i = base + uint64_t(j) * 256;
      if (i < vecs) v[j] = in[i];
    }
#pragma unroll
    for (int j = 0; j < kCopyUnroll; ++j) {
      const uint64_t i = base + uint64_t(j) * 256;
      if (i < vecs) out[i] = v[j];
    }
  }
}

__global__ void copy_tail_kernel(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, uint64_t bytes) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < bytes) out[i] = in[i];
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const T* __restrict__ in, uint64_t n_in, T* __restrict__ out,
                                                     const uint32_t* __restrict__ idx, uint64_t n) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n; j += stride) {
    const uint32_t s = idx[j];
    if (s < n_in) out[j] = in[s];
  }
}

// The random-read ceiling: each lane issues kRandomReads independent 4-byte
// loads at hashed word indices (all in flight at once), then one coalesced
// store of their sum, so nearly all traffic is random line fills.
constexpr int kRandomReads = 16;
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}
// T is the record read (4, 8 or 16 bytes); the sum of every record's first
// word is stored, so no load can be dropped.
__device__ __forceinline__ uint32_t first_word(uint32_t v) { return v; }
__device__ __forceinline__ uint32_t first_word(u32x2 v) { return v.x ^ v.y; }
__device__ __forceinline__ uint32_t first_word(u32x4 v) { return v.x ^ v.y ^ v.z ^ v.w; }
template <typename T>
__global__ __launch_bounds__(256) void random_reads_kernel(const T* __restrict__ in, uint32_t* __restrict__ out,
                                                           uint32_t mask, uint64_t lanes, uint32_t salt) {
  const uint64_t t = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  if (t >= lanes) return;
  T v[kRandomReads];
#pragma unroll
  for (int k = 0; k < kRandomReads; ++k) v[k] = in[hash32(uint32_t(t) * kRandomReads + k + salt) & mask];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kRandomReads; ++k) sum += first_word(v[k]);
  out[t] = sum;
}

int32_t g_probe_hip_error = 0;

}  // namespace

extern "C" {

bs_status bs_probe_copy(const void* in, void* out, uint64_t bytes, void* stream) {
  if (bytes == 0) return BS_OK;
  if (!in || !out) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % 16 || reinterpret_cast<uintptr_t>(out) % 16) return BS_EELEM;
  const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
  if (a < b + bytes && b < a + bytes) return BS_EALIAS;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t vecs = bytes / 16;
  if (vecs) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return BS_EHIP;
    const uint64_t want = (vecs + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
    const uint32_t grid = uint32_t(want < uint64_t(cus) * 8 ? want : uint64_t(cus) * 8);
    hipLaunchKernelGGL(copy16_kernel, dim3(grid), dim3(256), 0, s, static_cast<const u32x4*>(in),
                       static_cast<u32x4*>(out), vecs);
  }
  const uint64_t tail = bytes - vecs * 16;
  if (tail) {
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(64), 0, s, static_cast<const uint8_t*>(in) + vecs * 16,
                       static_cast<uint8_t*>(out) + vecs * 16, tail);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_probe_hip_error = int32_t(e);
    return BS_EHIP;
  }
  return BS_OK;
}

bs_status bs_probe_random_reads(const void* in, uint64_t words, void* out, uint32_t salt, void* stream) {
  return bs_probe_random_reads_region(in, words * 4, 4, words, out, salt, stream);
}

bs_status bs_probe_random_reads_region(const void* in, uint64_t region_bytes, uint32_t elem_bytes, uint64_t reads,
                                       void* out, uint32_t salt, void* stream) {
  if (!in || !out) return BS_EINVAL;
  if (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16) return BS_EELEM;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % 4) return BS_EELEM;
  const uint64_t records = region_bytes / elem_bytes;
  if (region_bytes % elem_bytes || records < 1 || records > (uint64_t(1) << 32) || (records & (records - 1)) != 0)
    return BS_EINVAL;
  if (reads < kRandomReads || reads % kRandomReads || reads / kRandomReads > (uint64_t(1) << 32)) return BS_EINVAL;
  const uint64_t lanes = reads / kRandomReads;
  const dim3 grid(uint32_t((lanes + 255) / 256));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t mask = uint32_t(records - 1);
  uint32_t* o = static_cast<uint32_t*>(out);
  switch (elem_bytes) {
    case 4:
      hipLaunchKernelGGL(random_reads_kernel<uint32_t>, grid, dim3(256), 0, s, static_cast<const uint32_t*>(in), o,
                         mask, lanes, salt);
      break;
    case 8:
      hipLaunchKernelGGL(random_reads_kernel<u32x2>, grid, dim3(256), 0, s, static_cast<const u32x2*>(in), o, mask,
                         lanes, salt);
      break;
    default:
      hipLaunchKernelGGL(random_reads_kernel<u32x4>, grid, dim3(256), 0, s, static_cast<const u32x4*>(in), o, mask,
                         lanes, salt);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_probe_hip_error = int32_t(e);
    return BS_EHIP;
  }
  return BS_OK;
}

bs_status bs_probe_gather(const void* in, uint64_t n_in, void* out, const uint32_t* idx, uint64_t n,
                          uint32_t elem_bytes, void* stream) {
  if (n == 0) return BS_OK;
  if (!in || !out || !idx) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(in) % elem_bytes || reinterpret_cast<uintptr_t>(out) % elem_bytes)
    return BS_EELEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t grid = uint32_t((n + 255) / 256 < 65536 * 4 ? (n + 255) / 256 : 65536 * 4);
  switch (elem_bytes) {
    case 1:
      hipLaunchKernelGGL(gather_kernel<uint8_t>, dim3(grid), dim3(256), 0, s, static_cast<const uint8_t*>(in), n_in,
                         static_cast<uint8_t*>(out), idx, n);
      break;
    case 2:
      hipLaunchKernelGGL(gather_kernel<uint16_t>, dim3(grid), dim3(256), 0, s, static_cast<const uint16_t*>(in),
                         n_in, static_cast<uint16_t*>(out), idx, n);
      break;
    case 4:
      hipLaunchKernelGGL(gather_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, static_cast<const uint32_t*>(in),
                         n_in, static_cast<uint32_t*>(out), idx, n);
      break;
    case 8:
      hipLaunchKernelGGL(gather_kernel<u32x2>, dim3(grid), dim3(256), 0, s, static_cast<const u32x2*>(in), n_in,
                         static_cast<u32x2*>(out), idx, n);
      break;
    case 16:
      hipLaunchKernelGGL(gather_kernel<u32x4>, dim3(grid), dim3(256), 0, s, static_cast<const u32x4*>(in), n_in,
                         static_cast<u32x4*>(out), idx, n);
      break;
    default:
      return BS_EELEM;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_probe_hip_error = int32_t(e);
    return BS_EHIP;
  }
  return BS_OK;
}

}  // extern "C"
