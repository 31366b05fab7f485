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

// Dependent round trips to device-coherent memory: lane 0 of every workgroup
// performs `chain` device-scope atomic adds in sequence, each address taken
// from the previous result (so none can start before the previous one
// returns), then stores the last result.  Timing launches of it against
// `chain` gives the cost of one round trip inside a small launch.
__global__ void round_trip_kernel(uint32_t* __restrict__ words, uint32_t chain) {
  if (threadIdx.x != 0) return;
  uint32_t x = 0;
  // x >> 31 is 0 for these counts, but the compiler cannot know it
  for (uint32_t i = 0; i < chain; ++i) x = atomicAdd(&words[(x >> 31) + blockIdx.x % 64u], 1u);
  words[64 + blockIdx.x % 64u] = x;
}

// Issue rate of one VALU instruction: 256 lanes per workgroup, eight
// independent chains per lane, `iters` instructions per chain, written in
// asm so the compiler neither fuses nor reorders them.  op: 0 v_xor_b32,
// 1 v_mul_u32_u24, 2 v_mad_u32_u24, 3 v_mul_lo_u32, 4 v_mul_hi_u32,
// 5 v_mad_u64_u32 (each followed by a v_xor_b32 of its two result words).
template <int OP>
__global__ __launch_bounds__(256) void int_rate_kernel(uint32_t* __restrict__ out, uint32_t iters, uint32_t c) {
  uint32_t a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 8u + uint32_t(j) + blockIdx.x;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if constexpr (OP == 0) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[j]) : "s"(c));
      if constexpr (OP == 1) asm volatile("v_mul_u32_u24 %0, %1, %0" : "+v"(a[j]) : "s"(c));
      if constexpr (OP == 2) asm volatile("v_mad_u32_u24 %0, %1, %0, %0" : "+v"(a[j]) : "s"(c));
      if constexpr (OP == 3) asm volatile("v_mul_lo_u32 %0, %1, %0" : "+v"(a[j]) : "s"(c));
      if constexpr (OP == 4) asm volatile("v_mul_hi_u32 %0, %1, %0" : "+v"(a[j]) : "s"(c));
      if constexpr (OP == 5) {
        uint64_t p, carry;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(p), "=s"(carry) : "s"(c), "v"(a[j]));
        a[j] = uint32_t(p) ^ uint32_t(p >> 32);
      }
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) x ^= a[j];
  out[blockIdx.x * 256u + threadIdx.x] = x;
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

bs_status bs_probe_int_rate(uint32_t op, uint32_t iters, uint32_t* out, uint32_t groups, void* stream) {
  if (!out || groups == 0 || groups > 65536 || iters == 0 || iters > (1u << 20) || op > 5) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(out) % 4) return BS_EELEM;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t c = 0x9E3779u;  // 24-bit multiplier: the 24-bit forms see the same operand
  switch (op) {
    case 0: hipLaunchKernelGGL(int_rate_kernel<0>, dim3(groups), dim3(256), 0, st, out, iters, c); break;
    case 1: hipLaunchKernelGGL(int_rate_kernel<1>, dim3(groups), dim3(256), 0, st, out, iters, c); break;
    case 2: hipLaunchKernelGGL(int_rate_kernel<2>, dim3(groups), dim3(256), 0, st, out, iters, c); break;
    case 3: hipLaunchKernelGGL(int_rate_kernel<3>, dim3(groups), dim3(256), 0, st, out, iters, c); break;
    case 4: hipLaunchKernelGGL(int_rate_kernel<4>, dim3(groups), dim3(256), 0, st, out, iters, c); break;
    default: hipLaunchKernelGGL(int_rate_kernel<5>, dim3(groups), dim3(256), 0, st, out, iters, c); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_probe_hip_error = int32_t(e);
    return BS_EHIP;
  }
  return BS_OK;
}

bs_status bs_probe_round_trips(uint32_t* words, uint32_t groups, uint32_t chain, void* stream) {
  if (!words || groups == 0 || groups > 65536 || chain > 1024) return BS_EINVAL;
  if (reinterpret_cast<uintptr_t>(words) % 4) return BS_EELEM;
  hipLaunchKernelGGL(round_trip_kernel, dim3(groups), dim3(64), 0, static_cast<hipStream_t>(stream), words, chain);
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
