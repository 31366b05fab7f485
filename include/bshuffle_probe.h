/*
 * bshuffle_probe.h -- measurement kernels exported by libbshuffle.so.
 *
 * These are not part of the shuffle.  They are the ceilings the shuffle's
 * throughput is reported against: the paper takes a random gather as the
 * upper bound of any GPU shuffle (Sec. 2.2, Sec. 6), and this library also
 * measures a plain device copy and the cipher-plus-scan work alone.
 * Pointers are device pointers on the current device; stream is a
 * hipStream_t as void*; returns as in bshuffle.h.
 */
#ifndef BSHUFFLE_PROBE_H
#define BSHUFFLE_PROBE_H

#include "bshuffle.h"

#ifdef __cplusplus
extern "C" {
#endif

/* out[0..bytes) = in[0..bytes) with 16-byte vector loads and stores.
 * in/out 16-byte aligned, non-overlapping. */
bs_status bs_probe_copy(const void *in, void *out, uint64_t bytes, void *stream);

/* The random-read ceiling: words/16 lanes each read 16 uint32 words of `in`
 * at hashed indices (hash of lane, read and salt, masked to words - 1), all
 * in flight at once, and write their sum to out[lane] (coalesced; out holds
 * words/16 uint32).  words is a power of two in [16, 2^32] (BS_EINVAL
 * otherwise); in and out 4-byte aligned (BS_EELEM).  Measures how many random
 * 4-byte reads per second the memory system serves, with almost no other
 * traffic. */
bs_status bs_probe_random_reads(const void *in, uint64_t words, void *out, uint32_t salt, void *stream);

/* The same ceiling over a chosen footprint and record size: `reads` random
 * reads of elem_bytes (4, 8 or 16; BS_EELEM otherwise) at hashed record
 * indices inside the first region_bytes of `in` (region_bytes / elem_bytes a
 * power of two in [1, 2^32]), 16 per lane, all in flight at once; out holds
 * reads/16 uint32 (one per lane).  reads is a multiple of 16, at most 2^36
 * (BS_EINVAL otherwise).  Separates the rate of random reads from the size of
 * the region they land in (caches, address translation) and from the bytes
 * each one carries.  bs_probe_random_reads(in, w, ...) is
 * bs_probe_random_reads_region(in, 4w, 4, w, ...). */
bs_status bs_probe_random_reads_region(const void *in, uint64_t region_bytes, uint32_t elem_bytes, uint64_t reads,
                                       void *out, uint32_t salt, void *stream);

/* Dependent round trips: `groups` workgroups of 64 lanes; lane 0 of each runs
 * `chain` device-scope atomic adds on words[0..64) in sequence (each address
 * depends on the previous result), then stores the last result in
 * words[64..128).  words: device memory of at least 128 uint32.  groups in
 * [1, 65536], chain <= 1024 (BS_EINVAL otherwise).  Timing it against `chain`
 * measures what one dependent global round trip costs a small launch (the
 * ticket, look-back and completion counters of a small shuffle are such
 * steps). */
bs_status bs_probe_round_trips(uint32_t *words, uint32_t groups, uint32_t chain, void *stream);

/* Issue rate of one integer VALU instruction: `groups` workgroups of 256
 * lanes, eight independent chains per lane of `iters` instructions each;
 * op 0 v_xor_b32, 1 v_mul_u32_u24, 2 v_mad_u32_u24, 3 v_mul_lo_u32,
 * 4 v_mul_hi_u32, 5 v_mad_u64_u32 (plus a v_xor_b32 of its result words).
 * out: device memory of groups * 256 uint32 (one word per lane, written so
 * the chains are not dropped).  groups in [1, 65536], iters in [1, 2^20],
 * op <= 5 (BS_EINVAL otherwise).  Timing a launch gives the cycles one wave
 * instruction of that kind holds a SIMD: the cipher's cost per round
 * (vp_round, vp_round_inverse) is counted in such instructions. */
bs_status bs_probe_int_rate(uint32_t op, uint32_t iters, uint32_t *out, uint32_t groups, void *stream);

/* Random gather with an index array: out[j] = in[idx[j]] for j < n, records
 * of elem_bytes (1,2,4,8,16); idx is a device uint32 array whose entries must
 * be < n_in (checked on the device: an out-of-range index is skipped). */
bs_status bs_probe_gather(const void *in, uint64_t n_in, void *out, const uint32_t *idx, uint64_t n,
                          uint32_t elem_bytes, void *stream);

/* The fused shuffle kernel with no payload: cipher, keep flags, wavefront
 * and workgroup scan, decoupled look-back; nothing is read or written but
 * the tile status words.  Same arguments and workspace rules as bs_shuffle. */
bs_status bs_probe_cipher_scan(uint64_t n, uint64_t seed, uint32_t rounds, void *workspace,
                               size_t workspace_bytes, void *stream);

/*
 * Less-fused forms of the same shuffle (Sec. 6's "Bijective1" and
 * "Bijective0"), for measurement; both write exactly bs_shuffle's output.
 *
 * bs_probe_shuffle_two_pass: the kept count of every tile first (cipher, no
 * payload), an exclusive scan of the counts, then the fused gather with known
 * tile prefixes (the cipher runs twice, no look-back).  n <= 2^32.
 *
 * bs_probe_shuffle_unfused: f over the whole padded domain written to a
 * table, a stream compaction of the images < n into a source list, then a
 * random gather through that list.  scratch: device memory of at least
 * bs_probe_unfused_scratch_bytes(n) bytes, 256-byte aligned.  n <= 2^32.
 */
bs_status bs_probe_shuffle_two_pass(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                                    uint32_t rounds, void *workspace, size_t workspace_bytes, void *stream);
size_t bs_probe_unfused_scratch_bytes(uint64_t n);
bs_status bs_probe_shuffle_unfused(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                                   uint32_t rounds, void *scratch, size_t scratch_bytes, void *workspace,
                                   size_t workspace_bytes, void *stream);

/*
 * bs_probe_set_watchdog -- failure-path testing of the look-back.  spin_limit:
 * polls after which a look-back wait gives up (0 restores the default, about
 * seconds of polling); the launch then records BS_ETIMEOUT for
 * bs_workspace_error, takes the nearest predecessor as a prefix of 0 and still
 * finishes, with every store kept inside `out`.  stall_first_tile = 1 makes
 * the first tile of every shuffle (and batch segment) withhold its status
 * word, so the next tile's wait deterministically runs into the limit; the
 * output is then wrong by design.  BS_EINVAL for stall_first_tile > 1.
 * Applies to every later launch from every thread.
 */
bs_status bs_probe_set_watchdog(uint32_t spin_limit, uint32_t stall_first_tile);

/*
 * bs_probe_set_xcd_mode -- how batched launches place segments on the 8 XCDs
 * (never changes results).  1: the batch's tiles are split into 8 ranges of
 * whole segments with about equal tile counts; workgroups take tiles from the
 * range of their own XCD first, so a segment's random reads stay in one L2.
 * 0: one range, tiles handed out in order to every XCD.  2 (default): ranges
 * when segments average at least 4 tiles.  BS_EINVAL for other values.
 * Applies to every later call from every thread.
 */
bs_status bs_probe_set_xcd_mode(uint32_t mode);

/*
 * bs_probe_set_batch_small -- how batched launches treat segments whose
 * padded domain has at most 2^10 indices (never changes results).  1
 * (default): one wavefront shuffles each such segment in registers, ranking
 * with its own ballots (no tile, no scan across wavefronts, no look-back), in
 * a second kernel after the tiled one.  0: every segment gets tiles.  BS_EINVAL
 * for other values.  Applies to every later call from every thread.
 */
bs_status bs_probe_set_batch_small(uint32_t enable);

/*
 * bs_probe_set_staged_policy -- when bs_shuffle takes the staged form (never
 * changes results): 0 never, 1 whenever the caller's workspace holds the
 * staged scratch (bs_workspace_bytes_staged) and the staged form covers n,
 * 2 (default) as the tuned table prefers.  BS_EINVAL for other values.
 * Applies to every later call from every thread.
 */
bs_status bs_probe_set_staged_policy(uint32_t mode);

/* Selects plain (0) or non-temporal (1) output stores for bs_shuffle. */
bs_status bs_probe_set_store_mode(uint32_t nontemporal);

#ifdef __cplusplus
}
#endif

#endif /* BSHUFFLE_PROBE_H */
