/*
 * oracle_sanitize_main.c -- drives the C oracle (oracle/cx_oracle.c) under
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).
 *
 * Random small collections (empty reads, duplicates, one-letter alphabets,
 * several thread counts) go through every exported oracle function: the
 * comparison sort, the BWT emit, the input validation and the invariant
 * checker on true and damaged BWTs.  The process exits 0 only if every
 * result is as expected; a sanitizer report aborts it.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int cx_oracle_validate(const uint8_t *text, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases);
int cx_oracle_sorted_suffixes(const uint8_t *text, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                              int threads, uint32_t *out_pairs);
int cx_oracle_bwt(const uint8_t *text, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases, int threads,
                  uint8_t *bwt, uint64_t *term_pos);
int cx_check_bwt(const uint8_t *bwt, const uint64_t *term_pos, const uint8_t *text, const uint64_t *offsets,
                 uint64_t n_reads, uint64_t n_bases, int threads);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t next_u32(void) { /* xorshift64* */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}
static uint32_t below(uint32_t k) { return next_u32() % k; }

static int failures = 0;
#define EXPECT(cond, what)                                         \
  do {                                                             \
    if (!(cond)) {                                                 \
      fprintf(stderr, "FAIL %s (trial %d)\n", what, trial);        \
      ++failures;                                                  \
    }                                                              \
  } while (0)

int main(void) {
  static const char alpha[] = "ACGT";
  for (int trial = 0; trial < 400; ++trial) {
    const uint64_t n = 1 + below(24);
    const uint32_t maxlen = below(4) == 0 ? 3 : 45;
    const uint32_t nsym = 1 + below(4);
    uint64_t *off = malloc(sizeof(uint64_t) * (n + 1));
    off[0] = 0;
    for (uint64_t i = 0; i < n; ++i) off[i + 1] = off[i] + below(maxlen + 1);
    const uint64_t nb = off[n];
    uint8_t *text = malloc(nb ? nb : 1);
    for (uint64_t t = 0; t < nb; ++t) text[t] = (uint8_t)alpha[below(nsym)];
    /* duplicate the first read over the second when both fit */
    if (n >= 2 && off[1] - off[0] <= off[2] - off[1] && below(2))
      memcpy(text + off[1], text + off[0], off[1] - off[0]);
    const uint64_t rows = nb + n;
    uint8_t *bwt = malloc(rows);
    uint64_t *tp = malloc(sizeof(uint64_t) * n);
    uint32_t *pairs = malloc(sizeof(uint32_t) * 2 * rows);
    const int threads = 1 + (int)below(4);
    EXPECT(cx_oracle_validate(text, off, n, nb) == 0, "validate accepts a valid collection");
    EXPECT(cx_oracle_bwt(text, off, n, nb, threads, bwt, tp) == 0, "bwt status");
    EXPECT(cx_oracle_sorted_suffixes(text, off, n, nb, threads, pairs) == 0, "sorted_suffixes status");
    EXPECT(cx_check_bwt(bwt, tp, text, off, n, nb, threads) == 0, "checker accepts the true BWT");
    /* rows 0..n-1 are the bare terminators in read order */
    for (uint64_t i = 0; i < n; ++i) EXPECT(pairs[2 * i] == i && pairs[2 * i + 1] == off[i + 1] - off[i], "bare rows");
    /* a damaged BWT: two rows of different symbols exchanged */
    uint64_t a = n + (rows > n ? below((uint32_t)(rows - n)) : 0), b = a;
    for (int k = 0; k < 64 && rows > n; ++k) {
      b = n + below((uint32_t)(rows - n));
      if (bwt[a] != bwt[b]) break;
    }
    if (rows > n && bwt[a] != bwt[b]) {
      uint8_t s = bwt[a];
      bwt[a] = bwt[b];
      bwt[b] = s;
      EXPECT(cx_check_bwt(bwt, tp, text, off, n, nb, threads) != 0, "checker rejects a damaged BWT");
    }
    /* invalid inputs are refused before any sorting */
    if (nb) {
      const uint8_t keep = text[nb - 1];
      text[nb - 1] = 'N';
      EXPECT(cx_oracle_validate(text, off, n, nb) != 0, "validate refuses a non-ACGT byte");
      EXPECT(cx_oracle_bwt(text, off, n, nb, threads, bwt, tp) != 0, "bwt refuses a non-ACGT byte");
      text[nb - 1] = keep;
    }
    if (n >= 2 && off[1] > 0) {
      const uint64_t keep = off[1];
      off[1] = off[2] + 1;
      EXPECT(cx_oracle_validate(text, off, n, nb) != 0, "validate refuses decreasing offsets");
      off[1] = keep;
    }
    free(pairs);
    free(tp);
    free(bwt);
    free(text);
    free(off);
  }
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("oracle sanitizer run ok\n");
  return 0;
}
