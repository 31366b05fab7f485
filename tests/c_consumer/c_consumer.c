/*
 * A plain C11 program that uses libbshuffle through its C ABI only (no
 * Python, no torch): device memory from the HIP runtime, bs_shuffle and
 * bs_shuffle_batched on the default stream, a caller-owned workspace, the
 * inverse through f^-1 and the bijection alone, and the error paths.  Results are checked against the sequential oracle
 * (test infrastructure, linked from oracle/liboracle.so).  Prints
 * "c_consumer: OK" and exits 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bshuffle.h"

/* oracle entry points (oracle/vphilox_oracle.c) */
int64_t orc_shuffle(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed, uint32_t rounds);
int orc_shuffle_batched(const void *in, void *out, const int64_t *offsets, const uint64_t *seeds,
                        uint32_t num_segments, uint32_t elem_bytes, uint32_t rounds);

#define CHECK_HIP(x)                                                   \
  do {                                                                 \
    hipError_t e_ = (x);                                               \
    if (e_ != hipSuccess) {                                            \
      fprintf(stderr, "%s:%d HIP error %d\n", __FILE__, __LINE__, e_); \
      return 1;                                                        \
    }                                                                  \
  } while (0)
#define CHECK_BS(x)                                                                          \
  do {                                                                                       \
    bs_status s_ = (x);                                                                      \
    if (s_ != BS_OK) {                                                                       \
      fprintf(stderr, "%s:%d %s (%d)\n", __FILE__, __LINE__, bs_status_string(s_), (int)s_); \
      return 1;                                                                              \
    }                                                                                        \
  } while (0)

static void fill(uint32_t *p, uint64_t n, uint64_t seed) {
  uint64_t s = seed;
  for (uint64_t i = 0; i < n; ++i) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    p[i] = (uint32_t)(s >> 32);
  }
}

int main(void) {
  const uint64_t n = 1000003;
  const uint32_t rounds = 24;
  uint32_t *h_in = malloc(n * 4), *h_out = malloc(n * 4), *want = malloc(n * 4);
  void *d_in = NULL, *d_out = NULL, *ws = NULL;
  if (!h_in || !h_out || !want) return 1;
  fill(h_in, n, 2106);
  CHECK_HIP(hipMalloc(&d_in, n * 4));
  CHECK_HIP(hipMalloc(&d_out, n * 4));
  CHECK_HIP(hipMemcpy(d_in, h_in, n * 4, hipMemcpyHostToDevice));

  /* one shuffle, library workspace cache, default stream */
  CHECK_BS(bs_shuffle(d_in, d_out, n, 4, 77, rounds, NULL, 0, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(h_out, d_out, n * 4, hipMemcpyDeviceToHost));
  if (orc_shuffle(h_in, want, n, 4, 77, rounds) != (int64_t)n || memcmp(h_out, want, n * 4) != 0) {
    fprintf(stderr, "bs_shuffle differs from the oracle\n");
    return 1;
  }

  /* five segments in one batched launch, caller-owned workspace */
  int64_t offsets[6] = {0, 1, 1000, 1000, 500000, (int64_t)n};
  uint64_t seeds[5] = {1, 2, 3, 4, 0xFFFFFFFFFFFFFFFFull};
  void *d_off = NULL, *d_seeds = NULL;
  const size_t ws_bytes = bs_workspace_bytes(n, 5, 4);
  CHECK_HIP(hipMalloc(&ws, ws_bytes));
  CHECK_BS(bs_workspace_init(ws, ws_bytes, NULL));
  CHECK_HIP(hipMalloc(&d_off, sizeof offsets));
  CHECK_HIP(hipMalloc(&d_seeds, sizeof seeds));
  CHECK_HIP(hipMemcpy(d_off, offsets, sizeof offsets, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_seeds, seeds, sizeof seeds, hipMemcpyHostToDevice));
  CHECK_BS(bs_shuffle_batched(d_in, d_out, d_off, d_seeds, 5, n, 4, rounds, ws, ws_bytes, NULL));
  CHECK_BS(bs_workspace_error(ws, NULL));
  CHECK_HIP(hipMemcpy(h_out, d_out, n * 4, hipMemcpyDeviceToHost));
  if (orc_shuffle_batched(h_in, want, offsets, seeds, 5, 4, rounds) != 0 || memcmp(h_out, want, n * 4) != 0) {
    fprintf(stderr, "bs_shuffle_batched differs from the oracle\n");
    return 1;
  }

  /* the inverse: gather form through f^-1 with caller scratch gives the input back */
  CHECK_BS(bs_shuffle(d_in, d_out, n, 4, 77, rounds, NULL, 0, NULL));
  void *d_back = NULL, *scratch = NULL;
  const size_t scratch_bytes = bs_unshuffle_inverse_scratch_bytes(n);
  CHECK_HIP(hipMalloc(&d_back, n * 4));
  CHECK_HIP(hipMalloc(&scratch, scratch_bytes));
  CHECK_BS(bs_unshuffle_inverse(d_out, d_back, n, 4, 77, rounds, scratch, scratch_bytes, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(h_out, d_back, n * 4, hipMemcpyDeviceToHost));
  if (memcmp(h_out, h_in, n * 4) != 0) {
    fprintf(stderr, "bs_unshuffle_inverse did not give the input back\n");
    return 1;
  }

  /* and through the staged streaming passes, with their own caller scratch */
  void *st_scratch = NULL;
  const size_t st_bytes = bs_unshuffle_staged_scratch_bytes(n, 4);
  CHECK_HIP(hipMalloc(&st_scratch, st_bytes));
  CHECK_HIP(hipMemset(d_back, 0, n * 4));
  CHECK_BS(bs_unshuffle_staged(d_out, d_back, n, 4, 77, rounds, st_scratch, st_bytes, NULL));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(h_out, d_back, n * 4, hipMemcpyDeviceToHost));
  if (memcmp(h_out, h_in, n * 4) != 0) {
    fprintf(stderr, "bs_unshuffle_staged did not give the input back\n");
    return 1;
  }
  CHECK_HIP(hipFree(st_scratch));

  /* the bijection alone: f then f^-1 is the identity on [0, 2^21) */
  enum { kVals = 4096 };
  uint64_t vals[kVals], back[kVals];
  for (int i = 0; i < kVals; ++i) vals[i] = ((uint64_t)i * 2654435761u) & ((1u << 21) - 1);
  void *d_vals = NULL;
  CHECK_HIP(hipMalloc(&d_vals, sizeof vals));
  CHECK_HIP(hipMemcpy(d_vals, vals, sizeof vals, hipMemcpyHostToDevice));
  CHECK_BS(bs_bijection(d_vals, d_vals, kVals, 21, 99, rounds, 0, NULL));
  CHECK_BS(bs_bijection(d_vals, d_vals, kVals, 21, 99, rounds, 1, NULL));
  CHECK_HIP(hipMemcpy(back, d_vals, sizeof back, hipMemcpyDeviceToHost));
  if (memcmp(back, vals, sizeof vals) != 0) {
    fprintf(stderr, "bs_bijection inverse did not undo the forward map\n");
    return 1;
  }
  CHECK_HIP(hipFree(d_vals));
  CHECK_HIP(hipFree(scratch));
  CHECK_HIP(hipFree(d_back));

  /* error paths are reported synchronously, nothing is launched */
  if (bs_shuffle(d_in, d_in, n, 4, 1, rounds, NULL, 0, NULL) != BS_EALIAS ||
      bs_shuffle(d_in, d_out, n, 3, 1, rounds, NULL, 0, NULL) != BS_EELEM ||
      bs_shuffle(d_in, d_out, n, 4, 1, BS_MAX_ROUNDS + 1, NULL, 0, NULL) != BS_EINVAL ||
      bs_shuffle(d_in, d_out, n, 4, 1, rounds, ws, 16, NULL) != BS_ENOMEM) {
    fprintf(stderr, "an argument error was not reported\n");
    return 1;
  }

  CHECK_HIP(hipFree(d_off));
  CHECK_HIP(hipFree(d_seeds));
  CHECK_HIP(hipFree(ws));
  CHECK_HIP(hipFree(d_in));
  CHECK_HIP(hipFree(d_out));
  free(h_in);
  free(h_out);
  free(want);
  printf("c_consumer: OK (libbshuffle %u)\n", bs_version());
  return 0;
}
