/*
 * cx_oracle.c -- plain CPU oracle for the multi-string Burrows-Wheeler
 * transform of a read collection (Liu, Luo & Lam, "GPU-Accelerated BWT
 * Construction for Large Collection of Short Reads", Section 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke entry point and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes (Section 2, the definition and Fig. 1):
 *   * Each read r_i (bases over A<C<G<T) is extended to S_i = r_i $_i.
 *   * The terminators sort below every base, and $_i < $_j exactly when i < j.
 *   * All sum_i (L_i + 1) suffixes S_i[k..], 0 <= k <= L_i, are sorted
 *     lexicographically; because every suffix ends in its own distinct $_i the
 *     order is strict and total, so exactly one answer exists.
 *   * Row rho of the BWT holds the symbol preceding the rho-th smallest
 *     suffix in its own string, or '$' when that suffix starts at offset 0.
 *   * term_pos[i] is the row of the offset-0 suffix of read i (the row whose
 *     BWT symbol is the '$' standing for read i).
 *
 * Variable read lengths (the paper fixes one length m) follow the same
 * definition with |S_i| = L_i + 1; empty reads (L_i = 0) are allowed and
 * contribute the single suffix $_i.
 *
 * Algorithm: the definition written out.  Every suffix is named by its
 * (read, offset) pair; the pairs are sorted with a comparison sort whose
 * comparator walks both suffixes symbol by symbol.  The sort is split over
 * threads (qsort per slice, then pairwise merges); the comparator decides a
 * strict total order, so the split cannot change the result.
 *
 * Parity status: pinned by tests (the Fig. 1 worked example, brute force over
 * explicit symbol tuples, the suffix array of the concatenated text with
 * distinct sentinels, closed forms and the LF-walk inverse).
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint32_t read; /* read index i */
  uint32_t off;  /* offset k inside read i, 0 <= k <= L_i */
} suffix_t;

typedef struct {
  const uint8_t *text;     /* reads concatenated, ASCII A/C/G/T */
  const uint64_t *offsets; /* n + 1 entries; read i = text[offsets[i], offsets[i+1]) */
} collection_t;

/* Rank of a base symbol in the alphabet order A < C < G < T (Section 2).
 * The terminator is handled separately (it ranks below every base). */
static int base_rank(uint8_t c) {
  switch (c) {
    case 'A': return 1;
    case 'C': return 2;
    case 'G': return 3;
    case 'T': return 4;
    default: return 99; /* never stored: inputs are validated first */
  }
}

/* Lexicographic comparison of S_a[ka..] and S_b[kb..] where S_i = r_i $_i. */
static int compare_suffixes(const void *pa, const void *pb, void *ctx) {
  const collection_t *c = (const collection_t *)ctx;
  const suffix_t *a = (const suffix_t *)pa;
  const suffix_t *b = (const suffix_t *)pb;
  const uint8_t *sa = c->text + c->offsets[a->read] + a->off;
  const uint8_t *sb = c->text + c->offsets[b->read] + b->off;
  uint64_t la = c->offsets[a->read + 1] - c->offsets[a->read] - a->off;
  uint64_t lb = c->offsets[b->read + 1] - c->offsets[b->read] - b->off;
  uint64_t t = 0;
  for (;; ++t) {
    int a_end = (t == la); /* suffix a shows its terminator at position t */
    int b_end = (t == lb);
    if (a_end && b_end) {
      /* both reach their terminators together: $_i < $_j iff i < j */
      return (a->read < b->read) ? -1 : (a->read > b->read) ? 1 : 0;
    }
    if (a_end) return -1; /* $ sorts below every base */
    if (b_end) return 1;
    int ra = base_rank(sa[t]);
    int rb = base_rank(sb[t]);
    if (ra != rb) return ra < rb ? -1 : 1;
  }
}

typedef struct {
  suffix_t *base;
  size_t count;
  const collection_t *coll;
} sort_job_t;

static void *sort_worker(void *p) {
  sort_job_t *j = (sort_job_t *)p;
  qsort_r(j->base, j->count, sizeof(suffix_t), compare_suffixes, (void *)j->coll);
  return NULL;
}

typedef struct {
  const suffix_t *left;
  size_t nleft;
  const suffix_t *right;
  size_t nright;
  suffix_t *dst;
  const collection_t *coll;
} merge_job_t;

static void *merge_worker(void *p) {
  merge_job_t *m = (merge_job_t *)p;
  size_t i = 0, j = 0, o = 0;
  while (i < m->nleft && j < m->nright) {
    if (compare_suffixes(&m->right[j], &m->left[i], (void *)m->coll) < 0)
      m->dst[o++] = m->right[j++];
    else
      m->dst[o++] = m->left[i++];
  }
  while (i < m->nleft) m->dst[o++] = m->left[i++];
  while (j < m->nright) m->dst[o++] = m->right[j++];
  return NULL;
}

/* Status codes of this oracle (independent of the library's own). */
#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -3

/*
 * cx_oracle_validate: 0 if text holds only A/C/G/T and offsets are a valid
 * non-decreasing partition of text with offsets[0] == 0; -1 otherwise.
 */
int cx_oracle_validate(const uint8_t *text, const uint64_t *offsets, uint64_t n_reads,
                       uint64_t n_bases) {
  if (n_reads > 0xFFFFFFFFull) return ORACLE_EINVAL;
  if (offsets[0] != 0 || offsets[n_reads] != n_bases) return ORACLE_EINVAL;
  for (uint64_t i = 0; i < n_reads; ++i) {
    if (offsets[i + 1] < offsets[i]) return ORACLE_EINVAL;
    if (offsets[i + 1] - offsets[i] > 0xFFFFFFFFull) return ORACLE_EINVAL;
  }
  for (uint64_t t = 0; t < n_bases; ++t)
    if (base_rank(text[t]) > 4) return ORACLE_EINVAL;
  return ORACLE_OK;
}

/*
 * cx_oracle_sorted_suffixes: sorted (read, offset) pairs, two uint32 per row,
 * written to out_pairs (2 * (n_bases + n_reads) entries).  threads <= 0 means 1.
 */
int cx_oracle_sorted_suffixes(const uint8_t *text, const uint64_t *offsets, uint64_t n_reads,
                              uint64_t n_bases, int threads, uint32_t *out_pairs) {
  int st = cx_oracle_validate(text, offsets, n_reads, n_bases);
  if (st != ORACLE_OK) return st;
  uint64_t total = n_bases + n_reads;
  if (total == 0) return ORACLE_OK;
  collection_t coll = {text, offsets};
  suffix_t *a = (suffix_t *)malloc(sizeof(suffix_t) * total);
  suffix_t *b = (suffix_t *)malloc(sizeof(suffix_t) * total);
  if (!a || !b) {
    free(a);
    free(b);
    return ORACLE_ENOMEM;
  }
  /* list every suffix (i, k), 0 <= k <= L_i */
  uint64_t row = 0;
  for (uint64_t i = 0; i < n_reads; ++i) {
    uint64_t len = offsets[i + 1] - offsets[i];
    for (uint64_t k = 0; k <= len; ++k) {
      a[row].read = (uint32_t)i;
      a[row].off = (uint32_t)k;
      ++row;
    }
  }
  if (threads <= 0) threads = 1;
  if ((uint64_t)threads > total) threads = (int)total;
  /* slice boundaries */
  size_t *cut = (size_t *)malloc(sizeof(size_t) * (threads + 1));
  for (int t = 0; t <= threads; ++t) cut[t] = (size_t)((total * (uint64_t)t) / (uint64_t)threads);
  pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * threads);
  sort_job_t *sj = (sort_job_t *)malloc(sizeof(sort_job_t) * threads);
  for (int t = 0; t < threads; ++t) {
    sj[t].base = a + cut[t];
    sj[t].count = cut[t + 1] - cut[t];
    sj[t].coll = &coll;
    pthread_create(&tid[t], NULL, sort_worker, &sj[t]);
  }
  for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
  /* pairwise merge rounds: runs [cut[s], cut[s+width]) */
  int runs = threads;
  size_t *rcut = cut;
  suffix_t *src = a, *dst = b;
  merge_job_t *mj = (merge_job_t *)malloc(sizeof(merge_job_t) * threads);
  while (runs > 1) {
    int pairs = runs / 2;
    for (int p = 0; p < pairs; ++p) {
      size_t l0 = rcut[2 * p], l1 = rcut[2 * p + 1], r1 = rcut[2 * p + 2];
      mj[p].left = src + l0;
      mj[p].nleft = l1 - l0;
      mj[p].right = src + l1;
      mj[p].nright = r1 - l1;
      mj[p].dst = dst + l0;
      mj[p].coll = &coll;
      pthread_create(&tid[p], NULL, merge_worker, &mj[p]);
    }
    if (runs % 2) { /* odd run out: copy through */
      size_t l0 = rcut[runs - 1], l1 = rcut[runs];
      memcpy(dst + l0, src + l0, sizeof(suffix_t) * (l1 - l0));
    }
    for (int p = 0; p < pairs; ++p) pthread_join(tid[p], NULL);
    /* new run boundaries */
    int nr = 0;
    for (int p = 0; p < pairs; ++p) rcut[nr++] = rcut[2 * p];
    if (runs % 2) rcut[nr++] = rcut[runs - 1];
    rcut[nr] = total;
    runs = nr;
    suffix_t *tmp = src;
    src = dst;
    dst = tmp;
  }
  for (uint64_t r = 0; r < total; ++r) {
    out_pairs[2 * r] = src[r].read;
    out_pairs[2 * r + 1] = src[r].off;
  }
  free(mj);
  free(sj);
  free(tid);
  free(cut);
  free(a);
  free(b);
  return ORACLE_OK;
}

/*
 * cx_oracle_bwt: the BWT (n_bases + n_reads ASCII bytes over A/C/G/T/$) and
 * term_pos (n_reads rows) of the collection.
 */
int cx_oracle_bwt(const uint8_t *text, const uint64_t *offsets, uint64_t n_reads,
                  uint64_t n_bases, int threads, uint8_t *bwt, uint64_t *term_pos) {
  uint64_t total = n_bases + n_reads;
  uint32_t *pairs = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (total ? total : 1));
  if (!pairs) return ORACLE_ENOMEM;
  int st = cx_oracle_sorted_suffixes(text, offsets, n_reads, n_bases, threads, pairs);
  if (st != ORACLE_OK) {
    free(pairs);
    return st;
  }
  for (uint64_t row = 0; row < total; ++row) {
    uint32_t i = pairs[2 * row], k = pairs[2 * row + 1];
    if (k == 0) {
      /* the suffix starts at offset 0: its preceding symbol is '$' */
      bwt[row] = '$';
      term_pos[i] = row;
    } else {
      bwt[row] = text[offsets[i] + k - 1];
    }
  }
  free(pairs);
  return ORACLE_OK;
}

/*
 * cx_check_bwt: the properties every multi-string BWT satisfies, checked in
 * O(N) memory for very large outputs (test infrastructure):
 *   1. symbol counts: the input bases plus one '$' per read;
 *   2. rows 0..n-1 are $_0..$_{n-1}: row i holds read i's last base ('$' if
 *      the read is empty);
 *   3. the LF walk from row i (LF(rho) = C[b] + #{rho' < rho : bwt[rho'] = b})
 *      spells read i backwards and stops on row term_pos[i] holding '$'.
 * Together these leave one possible string: the BWT.  Returns 0 when all
 * hold, otherwise a positive code naming the first property that failed.
 */
typedef struct {
  const uint8_t *bwt;
  const uint64_t *term_pos;
  const uint8_t *text;
  const uint64_t *offsets;
  const uint64_t *occ_base; /* per 64-row block: symbol counts before the block, 5 per block */
  uint64_t C[5];
  uint64_t r0, r1;          /* reads [r0, r1) */
  int failed;
} lf_job_t;

/* symbol code: 0 = '$', then A, C, G, T in their sort order; -1 for any other
 * byte (a table, filled once by cx_check_bwt before any worker starts) */
static signed char sym_table[256];

static void fill_sym_table(void) {
  static const char order[5] = {'$', 'A', 'C', 'G', 'T'};
  memset(sym_table, -1, sizeof(sym_table));
  for (int s = 0; s < 5; ++s) sym_table[(uint8_t)order[s]] = (signed char)s;
}

static inline int sym_code(uint8_t c) { return sym_table[c]; }

/* rank of symbol code s before row rho: block counts plus a scan inside the block */
static uint64_t occ_before(const lf_job_t *j, int s, uint64_t rho) {
  uint64_t blk = rho >> 6;
  uint64_t c = j->occ_base[blk * 5 + (uint64_t)s];
  for (uint64_t t = blk << 6; t < rho; ++t) c += (sym_code(j->bwt[t]) == s);
  return c;
}

static void *lf_worker(void *p) {
  lf_job_t *j = (lf_job_t *)p;
  for (uint64_t i = j->r0; i < j->r1 && !j->failed; ++i) {
    uint64_t a = j->offsets[i], b = j->offsets[i + 1];
    uint64_t rho = i; /* row of the bare terminator $_i */
    for (uint64_t step = 0;; ++step) {
      int s = sym_code(j->bwt[rho]);
      if (step == b - a) {
        if (s != 0 || j->term_pos[i] != rho) j->failed = 3;
        break;
      }
      uint8_t want = j->text[b - 1 - step];
      if (j->bwt[rho] != want) {
        j->failed = 3;
        break;
      }
      rho = j->C[s] + occ_before(j, s, rho);
    }
  }
  return NULL;
}

int cx_check_bwt(const uint8_t *bwt, const uint64_t *term_pos, const uint8_t *text, const uint64_t *offsets,
                 uint64_t n_reads, uint64_t n_bases, int threads) {
  uint64_t total = n_bases + n_reads;
  uint64_t cnt[5] = {0, 0, 0, 0, 0}, want[5] = {0, 0, 0, 0, 0};
  fill_sym_table();
  /* 1. counts */
  for (uint64_t t = 0; t < total; ++t) {
    int s = sym_code(bwt[t]);
    if (s < 0) return 1;
    cnt[s]++;
  }
  for (uint64_t t = 0; t < n_bases; ++t) {
    int s = sym_code(text[t]);
    if (s < 1) return 1;
    want[s]++;
  }
  want[0] = n_reads;
  for (int s = 0; s < 5; ++s)
    if (cnt[s] != want[s]) return 1;
  /* 2. bare-terminator rows */
  for (uint64_t i = 0; i < n_reads; ++i) {
    uint8_t w = offsets[i + 1] > offsets[i] ? text[offsets[i + 1] - 1] : (uint8_t)'$';
    if (bwt[i] != w) return 2;
  }
  /* 3. LF walks */
  uint64_t nblk = total / 64 + 1;
  uint64_t *occ = (uint64_t *)malloc(sizeof(uint64_t) * 5 * nblk);
  if (!occ) return ORACLE_ENOMEM;
  uint64_t run[5] = {0, 0, 0, 0, 0};
  for (uint64_t blk = 0; blk < nblk; ++blk) {
    for (int s = 0; s < 5; ++s) occ[blk * 5 + (uint64_t)s] = run[s];
    uint64_t t1 = (blk + 1) * 64 < total ? (blk + 1) * 64 : total;
    for (uint64_t t = blk * 64; t < t1; ++t) run[sym_code(bwt[t])]++;
  }
  if (threads <= 0) threads = 1;
  lf_job_t *jobs = (lf_job_t *)calloc((size_t)threads, sizeof(lf_job_t));
  pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * threads);
  uint64_t C[5];
  C[0] = 0;
  for (int s = 1; s < 5; ++s) C[s] = C[s - 1] + cnt[s - 1];
  for (int t = 0; t < threads; ++t) {
    jobs[t].bwt = bwt;
    jobs[t].term_pos = term_pos;
    jobs[t].text = text;
    jobs[t].offsets = offsets;
    jobs[t].occ_base = occ;
    memcpy(jobs[t].C, C, sizeof(C));
    jobs[t].r0 = n_reads * (uint64_t)t / (uint64_t)threads;
    jobs[t].r1 = n_reads * (uint64_t)(t + 1) / (uint64_t)threads;
    jobs[t].failed = 0;
    pthread_create(&tid[t], NULL, lf_worker, &jobs[t]);
  }
  int st = 0;
  for (int t = 0; t < threads; ++t) {
    pthread_join(tid[t], NULL);
    if (jobs[t].failed && !st) st = jobs[t].failed;
  }
  free(tid);
  free(jobs);
  free(occ);
  return st;
}
