/*
 * Sequential CPU oracle for the bijective shuffle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this file's library.  The product
 * path (the HIP library and its Python binding) never calls it, and the two
 * share no code: not the cipher, not the key schedule, not the compaction.
 *
 * What it computes (all integer, single thread, no blocking or fusion):
 *
 *  - The domain: the shuffle of n items runs a bijection on [0, 2^k) with
 *    k = max(ceil(log2 n), 4) (Sec. 4, padding to the nearest power of two;
 *    the floor of 4 is this project's reading, see orc_domain_bits).
 *
 *  - The round keys: the paper parameterises the shuffle by a key of
 *    rounds x log(n) bits but does not say how it is drawn (Sec. 7).  Here the
 *    r-th round key is the low 32 bits of the r-th output of SplitMix64
 *    (Steele, Lea and Flood, OOPSLA 2014) started from the 64-bit seed.
 *
 *  - VariablePhilox (Sec. 3.2, the text description of the cipher, its
 *    inverse, and the listing that fixes the arithmetic).  A k-bit block is
 *    split into a left half L of floor(k/2) bits, a right half R of the same
 *    width and, when k is odd, one extra bit b that sits between them:
 *        x = L | b | R      (L in the high bits, R in the low bits).
 *    One round, with the Philox constant M0 and the 64-bit product M0*L:
 *        F_key(L) = (high 32 bits of M0*L) xor key      (the round function)
 *        B(L)     =  low 32 bits of M0*L                 (a bijection mod 2^w)
 *        L'       = (F_key(L) xor R) restricted to the half width
 *        (R', b') = G(B(L), b): put b below the half-width B(L), then the top
 *                   bit of that (w+1)-bit word leaves as b' and the rest is R'.
 *    For even k there is no b and R' = B(L) restricted to the half width.
 *    The product M0*L is taken modulo 2^64 ("64 bit integer multiplication"),
 *    and B carries no key, as in the listing.
 *    The inverse runs the paper's three inversion steps in order:
 *        (B(L), b) = G^-1(R', b'),  L = B^-1(B(L)),  R = F_key(L) xor L'.
 *
 *  - Algorithm 1 (Sec. 4, "Bijection Shuffle"): for every i of the padded
 *    domain in increasing order, b = f(i); if b < n the element in[b] goes to
 *    the next free output slot.  The running count is the exclusive scan of
 *    the flags, so out[rank(i)] = in[f(i)].
 *
 * The linear congruential bijection of Sec. 3.1, y = (a*x + c) mod 2^k with a
 * odd, and Algorithm 1 run with it (the paper's low-quality comparison).
 *
 * Mallows-kernel helpers (Sec. 5): the number of discordant pairs n_dis of
 * two permutations, by brute force over all pairs and by merge-sort
 * inversion counting.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_ROUNDS 64
#define ORC_MIN_DOMAIN_BITS 4
#define ORC_MAX_DOMAIN_BITS 40

/* The Philox multiplier (Salmon et al. 2011) that the paper's VariablePhilox
 * uses. */
#define ORC_M0 0xD2B74407B1CE6E93ull

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2 };

typedef struct {
  uint32_t k;        /* domain bits: the cipher permutes [0, 2^k)        */
  uint32_t w;        /* half width: L and R each hold floor(k/2) bits     */
  uint32_t odd;      /* 1 when k is odd: the extra bit b exists           */
  uint32_t rounds;   /* number of Feistel rounds                          */
  uint32_t key[ORC_MAX_ROUNDS];
} orc_cipher;

/* ---------------------------------------------------------------- keys -- */

/* One SplitMix64 step: advance the state by the golden-ratio increment and
 * return the mixed value (published definition, constants 0x9E3779B97F4A7C15,
 * 0xBF58476D1CE4E5B9, 0x94D049BB133111EB with shifts 30, 27, 31). */
uint64_t orc_splitmix64_next(uint64_t *state) {
  uint64_t z;
  *state += 0x9E3779B97F4A7C15ull;
  z = *state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void orc_round_keys(uint64_t seed, uint32_t rounds, uint32_t *keys) {
  uint64_t st = seed;
  uint32_t r;
  for (r = 0; r < rounds; r++) keys[r] = (uint32_t)orc_splitmix64_next(&st);
}

/* ------------------------------------------------------------- domain -- */

/* Smallest k with 2^k >= n (0 for n <= 1). */
static uint32_t ceil_log2_u64(uint64_t n) {
  uint32_t k = 0;
  while (k < 64 && ((uint64_t)1 << k) < n) k++;
  return k;
}

/* Domain bits for a shuffle of n items: pad to the nearest power of two
 * (Sec. 4), but never below 2^4.  Below four bits the round is affine over
 * GF(2) with the key entering only as a translation, so the whole keyed family
 * holds at most 2^k permutations and could never pass the n=5 chi-square
 * test the paper reports (Sec. 5). */
uint32_t orc_domain_bits(uint64_t n) {
  uint32_t k = ceil_log2_u64(n);
  return k < ORC_MIN_DOMAIN_BITS ? ORC_MIN_DOMAIN_BITS : k;
}

/* Set up the cipher on [0, 2^k) for any k in [1, ORC_MAX_DOMAIN_BITS]; the
 * shuffle itself always uses orc_domain_bits(n).  Small k is allowed here so
 * the degeneracy argument above can be tested directly. */
int orc_cipher_init(orc_cipher *c, uint32_t k, uint64_t seed, uint32_t rounds) {
  if (!c || k < 1 || k > ORC_MAX_DOMAIN_BITS || rounds > ORC_MAX_ROUNDS)
    return ORC_EINVAL;
  memset(c, 0, sizeof(*c));
  c->k = k;
  c->w = k / 2;
  c->odd = k & 1u;
  c->rounds = rounds;
  orc_round_keys(seed, rounds, c->key);
  return ORC_OK;
}

/* ------------------------------------------------------------- cipher -- */

static uint64_t half_mask(uint32_t w) { return ((uint64_t)1 << w) - 1; }

/* The 64-bit product M0*L, split into its high and low 32-bit words. */
static void philox_product(uint32_t L, uint32_t *hi, uint32_t *lo) {
  uint64_t p = ORC_M0 * (uint64_t)L; /* modulo 2^64 */
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

/* F_key(L): the keyed, non-bijective round function. */
static uint64_t round_F(uint32_t L, uint32_t key, uint32_t w) {
  uint32_t hi, lo;
  philox_product(L, &hi, &lo);
  return (uint64_t)(hi ^ key) & half_mask(w);
}

/* B(L): the low word of the product, a bijection of w-bit values because M0
 * is odd. */
static uint64_t round_B(uint32_t L, uint32_t w) {
  uint32_t hi, lo;
  philox_product(L, &hi, &lo);
  return (uint64_t)lo & half_mask(w);
}

/* M0^-1 modulo 2^64 by Newton's iteration x <- x(2 - M0 x); each step doubles
 * the number of correct low bits, starting from 3 (M0*M0 = 1 mod 8). */
static uint64_t m0_inverse(void) {
  uint64_t x = ORC_M0;
  int i;
  for (i = 0; i < 6; i++) x *= 2 - ORC_M0 * x;
  return x;
}

uint64_t orc_encrypt(const orc_cipher *c, uint64_t x) {
  const uint32_t w = c->w;
  const uint64_t m = half_mask(w);
  uint64_t L, R, b;
  uint32_t r;
  /* x = L | b | R */
  R = x & m;
  b = c->odd ? (x >> w) & 1u : 0;
  L = (x >> (w + c->odd)) & m;
  for (r = 0; r < c->rounds; r++) {
    uint64_t Bv = round_B((uint32_t)L, w);
    uint64_t Lnew = round_F((uint32_t)L, c->key[r], w) ^ R;
    if (c->odd) {
      /* G: b enters below B(L); the word's top bit leaves as b'. */
      uint64_t g = (Bv << 1) | b;
      R = g & m;
      b = g >> w;
    } else {
      R = Bv;
    }
    L = Lnew;
  }
  return (L << (w + c->odd)) | (b << w) | R;
}

uint64_t orc_decrypt(const orc_cipher *c, uint64_t y) {
  const uint32_t w = c->w;
  const uint64_t m = half_mask(w);
  const uint64_t m0inv = m0_inverse();
  uint64_t L, R, b;
  uint32_t r;
  R = y & m;
  b = c->odd ? (y >> w) & 1u : 0;
  L = (y >> (w + c->odd)) & m;
  for (r = c->rounds; r-- > 0;) {
    /* Here (L, R, b) is the round's output (L', R', b'). */
    uint64_t Bv, Lprev;
    if (c->odd) {
      /* G^-1: rebuild the (w+1)-bit word; its low bit is the old b. */
      uint64_t g = (b << w) | R;
      b = g & 1u;
      Bv = g >> 1;
    } else {
      Bv = R;
    }
    Lprev = (Bv * m0inv) & m;                       /* B^-1 */
    R = round_F((uint32_t)Lprev, c->key[r], w) ^ L; /* R = F(L) xor L' */
    L = Lprev;
  }
  return (L << (w + c->odd)) | (b << w) | R;
}

/* f over the whole domain: table[x] = f(x) for x < 2^k.  k <= 32 only. */
int orc_encrypt_all(const orc_cipher *c, uint32_t *table) {
  uint64_t x, size;
  if (!c || !table || c->k > 32) return ORC_EINVAL;
  size = (uint64_t)1 << c->k;
  for (x = 0; x < size; x++) table[x] = (uint32_t)orc_encrypt(c, x);
  return ORC_OK;
}

/* ------------------------------------------------------------ shuffle -- */

static int check_shuffle_args(uint64_t n, uint32_t elem_bytes, uint32_t rounds) {
  if (elem_bytes == 0 || rounds > ORC_MAX_ROUNDS) return ORC_EINVAL;
  if (n > ((uint64_t)1 << ORC_MAX_DOMAIN_BITS)) return ORC_EINVAL;
  return ORC_OK;
}

/* Algorithm 1, run in index order from i = i_begin with `rank` outputs already
 * placed before it, stopping at i_end.  Returns the rank after i_end. */
static uint64_t shuffle_range(const orc_cipher *c, const uint8_t *in, uint8_t *out,
                              uint64_t n, uint32_t eb, uint64_t i_begin,
                              uint64_t i_end, uint64_t rank) {
  uint64_t i;
  for (i = i_begin; i < i_end; i++) {
    uint64_t src = orc_encrypt(c, i);
    if (src < n) { /* flag = 1: keep */
      if (out) memcpy(out + rank * eb, in + src * eb, eb);
      rank++;
    }
  }
  return rank;
}

/* out[rank(i)] = in[f(i)] for the n kept i.  Returns the number of items
 * written (always n) or a negative error. */
int64_t orc_shuffle(const void *in, void *out, uint64_t n, uint32_t elem_bytes,
                    uint64_t seed, uint32_t rounds) {
  orc_cipher c;
  uint64_t placed;
  if (check_shuffle_args(n, elem_bytes, rounds) != ORC_OK) return ORC_EINVAL;
  if (n == 0) return 0;
  if (!in || !out) return ORC_EINVAL;
  orc_cipher_init(&c, orc_domain_bits(n), seed, rounds);
  placed = shuffle_range(&c, (const uint8_t *)in, (uint8_t *)out, n, elem_bytes, 0,
                         (uint64_t)1 << c.k, 0);
  return (int64_t)placed;
}

/* The gather map itself: perm[j] = the input index that lands at output j. */
int64_t orc_shuffle_sources(uint64_t n, uint64_t seed, uint32_t rounds, uint64_t *perm) {
  orc_cipher c;
  uint64_t i, size, j = 0;
  if (check_shuffle_args(n, 1, rounds) != ORC_OK || (n && !perm)) return ORC_EINVAL;
  if (n == 0) return 0;
  orc_cipher_init(&c, orc_domain_bits(n), seed, rounds);
  size = (uint64_t)1 << c.k;
  for (i = 0; i < size; i++) {
    uint64_t src = orc_encrypt(&c, i);
    if (src < n) perm[j++] = src;
  }
  return (int64_t)j;
}

/* Number of kept indices in [i_begin, i_end): the exclusive scan of the flags
 * at i_end minus the one at i_begin. */
int64_t orc_count_kept(uint64_t n, uint64_t seed, uint32_t rounds, uint64_t i_begin,
                       uint64_t i_end) {
  orc_cipher c;
  if (check_shuffle_args(n, 1, rounds) != ORC_OK || n == 0) return ORC_EINVAL;
  orc_cipher_init(&c, orc_domain_bits(n), seed, rounds);
  if (i_end > ((uint64_t)1 << c.k)) i_end = (uint64_t)1 << c.k;
  if (i_begin > i_end) return ORC_EINVAL;
  return (int64_t)shuffle_range(&c, NULL, NULL, n, 1, i_begin, i_end, 0);
}

/* Outputs for the indices in [i_begin, i_end) only, given rank_begin = the
 * number of kept indices below i_begin.  Writes them to window[0..] and
 * returns how many were written.  Used to check a slice of a large shuffle. */
int64_t orc_shuffle_window(const void *in, uint64_t n, uint32_t elem_bytes, uint64_t seed,
                           uint32_t rounds, uint64_t i_begin, uint64_t i_end,
                           void *window) {
  orc_cipher c;
  uint64_t placed;
  if (check_shuffle_args(n, elem_bytes, rounds) != ORC_OK || n == 0 || !in || !window)
    return ORC_EINVAL;
  orc_cipher_init(&c, orc_domain_bits(n), seed, rounds);
  if (i_end > ((uint64_t)1 << c.k)) i_end = (uint64_t)1 << c.k;
  if (i_begin > i_end) return ORC_EINVAL;
  placed = shuffle_range(&c, (const uint8_t *)in, (uint8_t *)window, n, elem_bytes,
                         i_begin, i_end, 0);
  return (int64_t)placed;
}

/* Independent shuffles of packed segments: segment s is
 * in[offsets[s] .. offsets[s+1]) with its own seed, written to the same range
 * of out.  Each segment is exactly orc_shuffle of that slice. */
int orc_shuffle_batched(const void *in, void *out, const int64_t *offsets,
                        const uint64_t *seeds, uint32_t num_segments, uint32_t elem_bytes,
                        uint32_t rounds) {
  uint32_t s;
  if (!offsets || (num_segments && !seeds)) return ORC_EINVAL;
  for (s = 0; s < num_segments; s++) {
    int64_t a = offsets[s], e = offsets[s + 1];
    int64_t got;
    if (a < 0 || e < a) return ORC_EINVAL;
    got = orc_shuffle((const uint8_t *)in + (uint64_t)a * elem_bytes,
                      (uint8_t *)out + (uint64_t)a * elem_bytes, (uint64_t)(e - a),
                      elem_bytes, seeds[s], rounds);
    if (got != e - a) return ORC_EINVAL;
  }
  return ORC_OK;
}

/* ---------------------------------------------------- Mallows kernel -- */

/* n_dis(a, b) by definition: pairs i < j ordered one way by a and the other
 * way by b (Sec. 5).  O(n^2). */
uint64_t orc_discordant_pairs_brute(const uint32_t *a, const uint32_t *b, uint32_t n) {
  uint64_t d = 0;
  uint32_t i, j;
  for (i = 0; i < n; i++)
    for (j = i + 1; j < n; j++)
      if ((a[i] < a[j] && b[i] > b[j]) || (a[i] > a[j] && b[i] < b[j])) d++;
  return d;
}

static uint64_t merge_count(uint32_t *v, uint32_t *tmp, uint32_t lo, uint32_t hi) {
  uint32_t mid, i, j, k;
  uint64_t inv;
  if (hi - lo < 2) return 0;
  mid = lo + (hi - lo) / 2;
  inv = merge_count(v, tmp, lo, mid) + merge_count(v, tmp, mid, hi);
  i = lo; j = mid; k = lo;
  while (i < mid && j < hi) {
    if (v[i] <= v[j]) tmp[k++] = v[i++];
    else { inv += mid - i; tmp[k++] = v[j++]; }
  }
  while (i < mid) tmp[k++] = v[i++];
  while (j < hi) tmp[k++] = v[j++];
  memcpy(v + lo, tmp + lo, (size_t)(hi - lo) * sizeof(uint32_t));
  return inv;
}

/* n_dis(a, b) in O(n log n): reorder b by the positions that sort a, then
 * count inversions with merge sort.  a must hold distinct values < n. */
int64_t orc_discordant_pairs(const uint32_t *a, const uint32_t *b, uint32_t n) {
  uint32_t *order, *seq, *tmp;
  uint32_t i;
  uint64_t d;
  if (n < 2) return 0;
  order = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  seq = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  tmp = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
  if (!order || !seq || !tmp) { free(order); free(seq); free(tmp); return ORC_ENOMEM; }
  for (i = 0; i < n; i++) order[i] = UINT32_MAX;
  for (i = 0; i < n; i++) {
    if (a[i] >= n || order[a[i]] != UINT32_MAX) { free(order); free(seq); free(tmp); return ORC_EINVAL; }
    order[a[i]] = i;
  }
  for (i = 0; i < n; i++) seq[i] = b[order[i]];
  d = merge_count(seq, tmp, 0, n);
  free(order); free(seq); free(tmp);
  return (int64_t)d;
}

/* Sum over pairs (2i, 2i+1) of exp(-lambda * n_dis / C(n,2)) is done in
 * Python; this returns n_dis for each consecutive pair of rows of a
 * (num_perms x n) table. */
int orc_pair_discordances(const uint32_t *perms, uint64_t num_perms, uint32_t n,
                          uint64_t *out) {
  uint64_t p;
  for (p = 0; p + 1 < num_perms; p += 2) {
    int64_t d = orc_discordant_pairs(perms + p * n, perms + (p + 1) * n, n);
    if (d < 0) return (int)d;
    out[p / 2] = (uint64_t)d;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------ LCG bijection -- */

/* The linear congruential bijection of Sec. 3.1: y = (a*x + c) mod 2^k with
 * a odd (coprime to the power-of-two modulus).  Keyed from the seed: a is the
 * first SplitMix64 output forced odd, c the second, both reduced mod 2^k. */
void orc_lcg_params(uint64_t n, uint64_t seed, uint64_t *a, uint64_t *c) {
  uint64_t st = seed;
  const uint32_t k = orc_domain_bits(n);
  const uint64_t mask = (k >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << k) - 1);
  *a = (orc_splitmix64_next(&st) | 1u) & mask;
  *c = orc_splitmix64_next(&st) & mask;
}

/* Algorithm 1 with the LCG as the bijection: for i in increasing order, keep
 * y = (a*i + c) mod 2^k when y < n. */
int64_t orc_lcg_shuffle(const void *in, void *out, uint64_t n, uint32_t elem_bytes, uint64_t seed) {
  uint64_t a, c, i, size, mask, j = 0;
  uint32_t k;
  if (check_shuffle_args(n, elem_bytes, 0) != ORC_OK) return ORC_EINVAL;
  if (n == 0) return 0;
  if (!in || !out) return ORC_EINVAL;
  k = orc_domain_bits(n);
  size = (uint64_t)1 << k;
  mask = size - 1;
  orc_lcg_params(n, seed, &a, &c);
  for (i = 0; i < size; i++) {
    uint64_t y = (a * i + c) & mask;
    if (y < n) {
      memcpy((uint8_t *)out + j * elem_bytes, (const uint8_t *)in + y * elem_bytes, elem_bytes);
      j++;
    }
  }
  return (int64_t)j;
}
