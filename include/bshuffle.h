/*
 * bshuffle.h -- C ABI of the MI355X bijective-shuffle library (libbshuffle.so).
 *
 * The operation (Mitchell, Stokes, Frank, Holmes, "Bandwidth-Optimal Random
 * Shuffling for GPUs", arXiv 2106.06161):
 *
 *   - Sec. 4 and Algorithm 1 ("Bijection Shuffle"): to shuffle n items, pad
 *     the index range to a power of two 2^k, evaluate a keyed bijection f on
 *     every padded index i, keep the i whose image f(i) is < n, and give each
 *     kept i the output slot rank(i) = number of kept indices below i (an
 *     exclusive scan of the keep flags).  The result is
 *         out[rank(i)] = in[f(i)]      for every kept i.
 *     Here k = max(ceil(log2 n), 4).
 *   - Sec. 3.2 (VariablePhilox): f is a Feistel cipher on k-bit blocks with
 *     a Philox-style multiply round; `rounds` rounds, each with its own
 *     32-bit round key.  The paper recommends 24 rounds (Sec. 5).
 *   - Sec. 7: the shuffle is parameterised by the bijection and a key of
 *     rounds x log(n) bits.  This library derives the round keys from one
 *     64-bit seed: key r = low 32 bits of the r-th SplitMix64 output started
 *     at the seed.
 *
 * The output is a pure function of (input bytes, n, elem_bytes, seed, rounds):
 * launch configuration, workspace, stream and batching never change a byte.
 *
 * Conventions for every entry point:
 *   - Pointers named in/out/offsets/seeds/workspace are DEVICE pointers
 *     (hipMalloc / torch CUDA-tensor memory) on the current HIP device.
 *   - `stream` is a hipStream_t passed as void*; NULL means the legacy
 *     default stream.  Work is enqueued asynchronously on it; argument errors
 *     are returned synchronously before anything is enqueued, device-side
 *     problems are reported through bs_workspace_error().
 *   - No entry point throws; each returns a bs_status.
 *   - The caller owns every buffer it passes.  The library owns only its
 *     internal per-(device, stream) workspace cache, released at process exit.
 */
#ifndef BSHUFFLE_H
#define BSHUFFLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bs_status;

#define BS_OK 0        /* success                                              */
#define BS_EINVAL 1    /* null pointer, bad size, bad rounds or bad workspace  */
#define BS_EALIAS 2    /* in and out overlap (the method is out-of-place, Sec. 7) */
#define BS_EELEM 3     /* elem_bytes not in {1,2,4,8,16}, or a pointer not aligned to it */
#define BS_ENOMEM 4    /* workspace too small, or the internal cache could not grow */
#define BS_EHIP 5      /* a HIP runtime call or launch failed; see bs_last_hip_error() */
#define BS_ETIMEOUT 6  /* a look-back wait hit its spin limit (device side)     */
#define BS_ENODEV 7    /* no HIP device is available                           */
#define BS_EDEVICE 8   /* the device rejected the batch description (bad offsets, too many tiles) */

#define BS_MAX_ROUNDS 64u
/* Largest n: tile prefixes are packed into 38 bits of a status word. */
#define BS_MAX_ITEMS ((((uint64_t)1) << 38) - 1)
#define BS_MIN_DOMAIN_BITS 4u

/* Human-readable name of a status code (static storage). */
const char *bs_status_string(bs_status status);

/* The hipError_t value behind the most recent BS_EHIP on this thread (0 if none). */
int32_t bs_last_hip_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
uint32_t bs_version(void);

/* k = max(ceil(log2 n), 4): the cipher runs on [0, 2^k) (Sec. 4 padding). */
uint32_t bs_domain_bits(uint64_t n);

/* Writes keys[r] = low 32 bits of the r-th SplitMix64 output from `seed`,
 * r < rounds (host memory).  Exposed so callers can see the key schedule. */
bs_status bs_round_keys(uint64_t seed, uint32_t rounds, uint32_t *keys);

/*
 * Workspace needed by one call: a 256-byte header plus one 8-byte status word
 * per tile of the padded domain, plus (batched) per-segment tables.
 *   single call : bs_workspace_bytes(n, 0, elem_bytes)
 *   batched call: bs_workspace_bytes(total_items, num_segments, elem_bytes),
 *                 total_items = offsets[num_segments].
 * The figure is an upper bound for every launch configuration.
 */
size_t bs_workspace_bytes(uint64_t items, uint32_t num_segments, uint32_t elem_bytes);

/*
 * Prepares caller-owned workspace memory for first use: zero-fills it and
 * records its capacity, asynchronously on `stream`.  A workspace must be
 * initialised once (or zero-filled by the caller) before its first use; the
 * library keeps it consistent afterwards.  Two calls whose executions overlap
 * in time must not share a workspace.
 */
bs_status bs_workspace_init(void *workspace, size_t workspace_bytes, void *stream);

/*
 * Reads and clears the workspace's sticky device-side error word.  Blocks
 * until `stream` has drained.  Returns BS_OK, BS_ETIMEOUT or BS_EDEVICE.
 * workspace == NULL inspects the library's own workspace for (device, stream).
 */
bs_status bs_workspace_error(void *workspace, void *stream);

/*
 * The same, without blocking: enqueues on `stream` a one-thread kernel that
 * writes BS_OK, BS_ETIMEOUT or BS_EDEVICE to *status and clears the
 * workspace's error word, so the status covers exactly the work enqueued on
 * `stream` since the previous read.  `status` is device-writable memory (a
 * device buffer, or pinned host memory from hipHostMalloc) of 4 bytes,
 * 4-byte aligned; it holds the result once the stream has reached this point
 * (an event recorded after this call has completed).  `workspace` is a
 * caller's workspace (256-byte aligned; there is no NULL form).  BS_EINVAL for
 * null or misaligned pointers.  Capturable in a graph.  Serving loops use it
 * to fail exactly the launch whose look-back timed out or whose batch was
 * malformed (Algorithm 1's scan is the step that can report either).
 */
bs_status bs_workspace_error_async(void *workspace, int32_t *status, void *stream);

/*
 * bs_shuffle -- one bijective shuffle (Algorithm 1, fused in a single pass).
 *
 *   in, out     device buffers of n records of elem_bytes bytes each; they
 *               must not overlap (BS_EALIAS) and must be aligned to
 *               elem_bytes (BS_EELEM).  Records are moved as raw bytes, so
 *               any payload type is bit-exact.
 *   n           number of records, 0 <= n <= BS_MAX_ITEMS; n = 0 is a no-op.
 *   elem_bytes  1, 2, 4, 8 or 16.
 *   seed        any 64-bit value; selects the round keys.
 *   rounds      0..64.  0 gives the identity permutation (out = in).
 *   workspace   device memory of workspace_bytes >= bs_workspace_bytes(n,0,eb)
 *               prepared by bs_workspace_init, or NULL to use the library's
 *               per-(device, stream) cache (grown with hipMalloc when needed).
 *               A call captured into a graph must pass its own workspace
 *               (NULL while `stream` is capturing returns BS_EINVAL: a later
 *               call could regrow the cache under the captured graph).
 *   stream      hipStream_t as void*.
 *
 * Writes out[rank(i)] = in[f(i)] for every padded index i < 2^k with f(i) < n.
 */
bs_status bs_shuffle(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                     uint32_t rounds, void *workspace, size_t workspace_bytes, void *stream);

/*
 * bs_shuffle_noalloc -- bs_shuffle for callers that cannot allocate device
 * memory (code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc): the same result byte for byte, with no
 * workspace argument.  Its kernels keep their tile status words and counters
 * in a device array of static storage inside the library, one per GPU,
 * BS_NOALLOC_SCRATCH_BYTES bytes (about 4 MiB), held until the process ends.
 * No hipMalloc, hipFree or other allocating routine is ever called.
 *
 *   in, out, elem_bytes, seed, rounds, stream   as for bs_shuffle.
 *   n           0 <= n <= BS_NOALLOC_MAX_ITEMS (2^30); larger n returns
 *               BS_ENOMEM (the array is too small) and enqueues nothing.
 *
 * The first call on a device looks up that device's array and zero-fills it
 * on `stream`; that first call must not be made while `stream` is capturing
 * (BS_EINVAL): make one call outside capture first.  Later calls, captured
 * or not, need nothing more: each launch leaves the array ready for the next.
 * All calls on one GPU share its array, so two bs_shuffle_noalloc calls whose
 * executions overlap on one GPU (different streams, or graphs replayed
 * concurrently) race and give wrong results; serialize them.  Device-side
 * errors are sticky in the array; there is no entry point to read them, so
 * callers that need the look-back watchdog's report use bs_shuffle.
 */
#define BS_NOALLOC_MAX_ITEMS (((uint64_t)1) << 30)
#define BS_NOALLOC_SCRATCH_BYTES (256u + (1u << 19) * 8u)
bs_status bs_shuffle_noalloc(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                             uint32_t rounds, void *stream);

/*
 * bs_shuffle_batched -- many independent shuffles in one launch sequence.
 *
 *   offsets     device int64[num_segments + 1], offsets[0] = 0, non-decreasing;
 *               segment s is records [offsets[s], offsets[s+1]) of in and out.
 *   seeds       device uint64[num_segments]: the seed of each segment.
 *   total_items offsets[num_segments] (host copy; sizes the launch).
 *   Other arguments as for bs_shuffle; one elem_bytes and one round count
 *   for the whole batch.
 *
 * Segment s of out equals bs_shuffle of segment s of in with seeds[s],
 * byte for byte.  A malformed offsets array is detected on the device: no
 * byte of out is written and bs_workspace_error() reports BS_EDEVICE.
 */
bs_status bs_shuffle_batched(const void *in, void *out, const int64_t *offsets,
                             const uint64_t *seeds, uint32_t num_segments, uint64_t total_items,
                             uint32_t elem_bytes, uint32_t rounds, void *workspace,
                             size_t workspace_bytes, void *stream);

/*
 * bs_permutation -- the permutation itself: out_idx[j] = the input position
 * of the record that bs_shuffle(n, seed, rounds) puts at output j, i.e. f(i)
 * for the j-th kept padded index (Algorithm 1 with the index as payload).
 * index_bytes is 4 (n <= 2^32) or 8; out_idx is a device array of n indices
 * aligned to index_bytes.  Workspace and stream as for bs_shuffle.
 */
bs_status bs_permutation(void *out_idx, uint64_t n, uint32_t index_bytes, uint64_t seed, uint32_t rounds,
                         void *workspace, size_t workspace_bytes, void *stream);

/*
 * bs_unshuffle -- the inverse of bs_shuffle with the same (n, seed, rounds):
 * out[f(i)] = in[rank(i)] for every kept padded index i (VariablePhilox is
 * a bijection, Sec. 3.2; its inverse permutation undoes the shuffle), so
 * bs_unshuffle(bs_shuffle(x)) == x.  Reads are coalesced, writes scattered.
 * Arguments and errors as for bs_shuffle.  bs_unshuffle_staged computes the
 * same output with streaming passes only (below).
 */
bs_status bs_unshuffle(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed, uint32_t rounds,
                       void *workspace, size_t workspace_bytes, void *stream);

/*
 * bs_unshuffle_inverse -- the same result as bs_unshuffle, computed in gather
 * form through the inverse cipher (Sec. 3.2): for every output position
 * p < n, i = f^-1(p) is the padded index whose image is p, and
 * out[p] = in[rank(i)], rank(i) being the number of kept indices below i.
 * The ranks come from a table built in one pass over the padded domain (a
 * 32-bit mask of kept flags and a 32-bit count per 32 indices, plus one
 * 64-bit count and prefix per 8192 indices), kept in `scratch`.  Writes are
 * coalesced; each output reads one table entry and one record at random.
 *
 *   scratch  device memory of at least bs_unshuffle_inverse_scratch_bytes(n)
 *            bytes (about 2^k / 4 bytes for the domain 2^k), 256-byte aligned,
 *            overlapping neither in nor out; its contents on entry do not
 *            matter and are overwritten.  NULL or misaligned: BS_EINVAL; too
 *            small: BS_ENOMEM.
 * Other arguments and errors as for bs_unshuffle.  No workspace: there is no
 * look-back.  bs_unshuffle_inverse_scratch_bytes returns 0 for n > BS_MAX_ITEMS.
 */
size_t bs_unshuffle_inverse_scratch_bytes(uint64_t n);
bs_status bs_unshuffle_inverse(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                               uint32_t rounds, void *scratch, size_t scratch_bytes, void *stream);

/*
 * bs_shuffle_staged -- exactly bs_shuffle's output, out[rank(i)] = in[f(i)],
 * computed by streaming passes instead of random gathers.  Algorithm 1 seen
 * from the input side sends record y < n to position rank(f^-1(y)), f^-1
 * being the inverse cipher (Sec. 3.2).  The input is read in order; each
 * record goes with its padded index i = f^-1(y) into buckets by the high bits
 * of i (one or two distribution passes through LDS, whole cache lines to and
 * from memory); one workgroup per window of 2^s consecutive padded indices
 * then places the window's records by rank (a popcount over the window's
 * kept indices plus the kept count of earlier windows) and writes them in
 * order.  Memory traffic per record: elem_bytes read and elem_bytes + 4
 * written by the first pass, elem_bytes + 4 read and elem_bytes + 2 written
 * by the second, elem_bytes + 2 read and elem_bytes written by the place
 * pass (6 * elem_bytes + 12 in all; 36 bytes for 4-byte records), every
 * access part of a whole-line stream, against one random 128-byte line fill
 * per record in bs_shuffle.
 *
 *   scratch  device memory of at least bs_staged_scratch_bytes(n, elem_bytes)
 *            bytes, 256-byte aligned, overlapping neither in nor out: about
 *            2^k * (2 * elem_bytes + 6) bytes for the padded domain 2^k (one
 *            bucket array per distribution pass, each with room for every
 *            padded index so no bucket can overflow; 4-byte indices in the
 *            first, 2-byte window indices in the second).  Contents on entry
 *            do not matter.  NULL or misaligned: BS_EINVAL; too small:
 *            BS_ENOMEM; overlapping in or out: BS_EALIAS.
 * Covers padded domains up to 2^32 (and elem_bytes 16 up to 2^30, 8 up to
 * 2^31): bs_staged_scratch_bytes returns 0 and bs_shuffle_staged BS_EINVAL
 * outside them.  Other arguments and errors as for bs_shuffle; there is no
 * look-back (the passes are ordered by the stream) and no workspace.
 */
size_t bs_staged_scratch_bytes(uint64_t n, uint32_t elem_bytes);

/*
 * bs_workspace_bytes_staged -- a workspace size with which bs_shuffle may take
 * the staged form: bs_workspace_bytes(n, 0, elem_bytes) rounded up to 256
 * bytes, plus bs_staged_scratch_bytes(n, elem_bytes) (just the former when
 * the staged form does not cover n).  bs_shuffle runs the staged form, with
 * the same output, when its caller-provided workspace is at least this large
 * and the tuned table prefers the staged form for the call's element size and
 * domain bits (a "staged" table line; see bs_autotune); otherwise, and always
 * with the library's own workspace or while a shape is forced with
 * bs_set_config, it runs the fused kernel.  0 for n > BS_MAX_ITEMS or a bad
 * elem_bytes.
 */
size_t bs_workspace_bytes_staged(uint64_t n, uint32_t elem_bytes);
bs_status bs_shuffle_staged(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                            uint32_t rounds, void *scratch, size_t scratch_bytes, void *stream);

/*
 * bs_unshuffle_staged -- exactly bs_unshuffle's output, out[f(i)] = in[rank(i)]
 * for every kept padded index i (the inverse permutation of the shuffle,
 * Sec. 3.2 and Algorithm 1), computed by streaming passes instead of
 * scattered writes: per tile of padded indices the forward cipher and the
 * kept images f(i) in index order; a scan of the tiles' kept counts (a
 * tile's records are then the consecutive in[] entries from its first rank);
 * the images with their records distributed into buckets by the high bits
 * of f(i), as bs_shuffle_staged distributes by i; and the place pass, where
 * the positions f(i) fill every slot below n, so each window is written in
 * order.  Memory traffic per record: the kept images written and read (4 + 4),
 * then bs_shuffle_staged's passes (6 * elem_bytes + 12).
 *
 *   scratch  device memory of at least bs_unshuffle_staged_scratch_bytes(n,
 *            elem_bytes) bytes: bs_staged_scratch_bytes plus 4 bytes per
 *            padded index and 8 per tile of padded indices; other conditions
 *            and errors as for bs_shuffle_staged.
 * Covers the domains bs_shuffle_staged covers (bs_unshuffle_staged_scratch_bytes
 * returns 0 and bs_unshuffle_staged BS_EINVAL outside them).
 */
size_t bs_unshuffle_staged_scratch_bytes(uint64_t n, uint32_t elem_bytes);
bs_status bs_unshuffle_staged(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                              uint32_t rounds, void *scratch, size_t scratch_bytes, void *stream);

/*
 * The linear congruential bijection of Sec. 3.1 as the shuffle's f, for
 * comparison with VariablePhilox (Sec. 5 reports its poor quality: at n = 5
 * its chi-square statistic is in the hundreds of thousands).
 *
 * bs_lcg_params -- the LCG of a call: f(x) = (a*x + c) mod 2^k with
 * k = bs_domain_bits(n), a = (first SplitMix64 output of seed) | 1 and
 * c = second output, both reduced mod 2^k.  Host only; BS_EINVAL for null
 * pointers or n > BS_MAX_ITEMS.
 *
 * bs_shuffle_lcg -- Algorithm 1 with that f: out[rank(i)] = in[f(i)] over the
 * kept padded indices i, in one fused pass as bs_shuffle.  Arguments, workspace
 * and errors as for bs_shuffle (there are no rounds).
 */
bs_status bs_lcg_params(uint64_t n, uint64_t seed, uint64_t *a, uint64_t *c);
bs_status bs_shuffle_lcg(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed, void *workspace,
                         size_t workspace_bytes, void *stream);

/*
 * bs_bijection -- the keyed bijection alone, applied elementwise: with
 * inverse = 0, out[j] = f(in[j]); with inverse = 1, out[j] = f^-1(in[j]),
 * where f is VariablePhilox on [0, 2^domain_bits) with the round keys of
 * `seed` (Sec. 3.2: the cipher and the three steps that invert it).  For
 * domain_bits = bs_domain_bits(n), f is the map that bs_shuffle(n, seed,
 * rounds) applies to padded indices.  Each in[j] is reduced mod
 * 2^domain_bits first.  in and out are device arrays of `count` uint64_t,
 * 8-byte aligned (BS_EELEM otherwise); in == out is allowed, other overlap
 * is not.  domain_bits in [1, BS_MAX_BIJECTION_BITS], rounds <=
 * BS_MAX_ROUNDS, inverse 0 or 1 (BS_EINVAL otherwise).  No workspace;
 * asynchronous on `stream`; count == 0 does nothing.
 */
#define BS_MAX_BIJECTION_BITS 40u
bs_status bs_bijection(const uint64_t *in, uint64_t *out, uint64_t count, uint32_t domain_bits, uint64_t seed,
                       uint32_t rounds, uint32_t inverse, void *stream);

/*
 * Launch configuration (never changes results).  A tile is waves x 64 x items
 * padded indices; depth selects the tile schedule: 1 or 2 tiles in flight per
 * workgroup with the kept records held in registers; BS_DEPTH_COMPACT, where a
 * tile's kept images are first compacted in LDS and then gathered and stored
 * by all lanes in rank order; or BS_DEPTH_COMPACT_PIPE, the same with the next
 * tile's cipher computed while the current tile's gathers are in flight.
 * Single shuffles whose domain needs 64-bit indices (k > 32) always run the
 * pipelined compacted schedule with 16 waves x 8 items, whatever shape is
 * configured.
 * Compiled shapes (waves, items, depth): (4,16,2) (8,16,2) (8,16,1)
 * (16,16,1) (16,8,1) (8,8,2) (4,16,1) (16,16,2) (16,8,2), and with either
 * compacted schedule (16,16) (8,16) (16,8) (8,8) (4,16).  grid_mult: 0 = a persistent grid of
 * as many workgroups as the device keeps resident, 1..64 = that many
 * workgroups per CU, BS_GRID_ONE_PER_TILE = one workgroup per tile.
 * bs_set_config with a shape forces it for every later call (from every
 * thread), ignoring the tuned table; bs_set_config(0, 0, 0, 0) restores the
 * default and re-enables the tuned table.  BS_EINVAL for a shape that is not
 * compiled.
 */
#define BS_GRID_ONE_PER_TILE 1000u
#define BS_DEPTH_COMPACT 8u
#define BS_DEPTH_COMPACT_PIPE 9u
/* bs_query_config's depth for a bs_shuffle that takes the staged form
 * (bs_shuffle_staged's passes; waves and items are then 0). */
#define BS_DEPTH_STAGED 16u
bs_status bs_set_config(uint32_t waves_per_group, uint32_t items_per_lane, uint32_t depth, uint32_t grid_mult);
bs_status bs_get_config(uint32_t *waves_per_group, uint32_t *items_per_lane, uint32_t *depth,
                        uint32_t *grid_mult);

/*
 * Tuned launch shapes (filled by bs_autotune or a table file; never change results).
 * kind 0 = bs_shuffle, keyed by the domain bits k of the call; kind 1 =
 * bs_shuffle_batched, keyed by ceil(log2(mean segment size)).  Unless a shape
 * was forced with bs_set_config, a call uses the entry for (kind, elem_bytes,
 * size class), else the nearest tuned class of that kind and element size
 * (the largest below, then the smallest above), else the default shape.
 */
bs_status bs_set_tuned_config(uint32_t kind, uint32_t elem_bytes, uint32_t size_bits, uint32_t waves_per_group,
                              uint32_t items_per_lane, uint32_t depth, uint32_t grid_mult);
bs_status bs_clear_tuned_configs(void);

/*
 * Native autotuner and tuned-table files (text; see the format below).
 *
 * bs_autotune -- if cache_path names a table made for the architecture of
 * `device`, loads it; otherwise times every compiled shape and grid choice on
 * `device` for every element size (single shuffles with domains of
 * 2^12 .. 2^max_size_bits indices, batched launches with mean segment sizes
 * of 2^8 .. 2^min(20, max_size_bits)), installs the fastest per size class
 * and, when cache_path is not NULL, writes the table there.  max_size_bits 0
 * means 30.  flags: 0, or BS_AUTOTUNE_VERBOSE for one line on stderr per tuned
 * size class.  Tuning allocates its own buffers (at most half the free device
 * memory, 40 GiB at most) and a stream, takes minutes at the default sizes,
 * and restores any shape forced with bs_set_config.  BS_ENODEV without a
 * device, BS_EINVAL for a bad device index, unknown flags or an unwritable
 * cache_path.
 *
 * bs_load_tuned_configs -- replaces the tuned table with the file's entries
 * (the arch line is not checked).  BS_EINVAL if the file cannot be read or an
 * entry is malformed or names a shape that is not compiled; the table is then
 * unchanged.
 *
 * bs_save_tuned_configs -- writes the current tuned table, with the current
 * device's architecture when one is available.
 *
 * Format: '#' starts a comment; "arch <name>" and "rounds <r>" lines; one
 * entry per line: kind elem_bytes size_bits waves items depth grid_mult [ms],
 * or "staged elem_bytes size_bits prefer [ms_staged ms_fused]" (prefer = 1:
 * bs_shuffle takes the staged form for that class when its workspace allows,
 * see bs_workspace_bytes_staged).  The tuner times the staged form against
 * the best fused shape for single-shuffle classes of 2^20 indices and up.
 * Like the shapes, a class without an entry takes the nearest listed class
 * of the same element size below it (so domains above the largest tuned
 * class keep its choice); below the smallest listed class, the fused form.
 */
#define BS_AUTOTUNE_VERBOSE 1u
bs_status bs_autotune(int device, const char *cache_path, uint32_t max_size_bits, uint32_t flags);
bs_status bs_load_tuned_configs(const char *path);
bs_status bs_save_tuned_configs(const char *path);

/* The launch shape a call would use: kind 0 = bs_shuffle of `items` records,
 * kind 1 = bs_shuffle_batched of `items` records in num_segments segments. */
bs_status bs_query_config(uint32_t kind, uint32_t elem_bytes, uint64_t items, uint32_t num_segments,
                          uint32_t *waves_per_group, uint32_t *items_per_lane, uint32_t *depth,
                          uint32_t *grid_mult);

#ifdef __cplusplus
}
#endif

#endif /* BSHUFFLE_H */
