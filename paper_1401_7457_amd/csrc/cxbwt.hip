// cxbwt.hip -- multi-string BWT of a read collection on MI355X (gfx950).
//
// Liu, Luo & Lam, "GPU-Accelerated BWT Construction for Large Collection of
// Short Reads": Section 2 defines the transform (sort every suffix of every
// S_i = r_i $_i, terminators below the bases and ordered by read index, emit
// the preceding symbol); Section 3.2 sorts suffixes with LSD radix passes over
// packed 2-bit "stringwords" gathered by index, with '$' padding and stable
// passes giving the read-index tie-break.
//
// This implementation keeps the idea of sorting suffix handles by packed
// multi-base keys gathered from the 2-bit reads, but organises the sort for a
// 256-CU, 8 TB/s device:
//
//   * handle  = the 32-bit global base position p of a suffix's first base;
//               the n empty suffixes ($_i alone) are not sorted at all: they
//               are rows 0..n-1 in read order.
//   * key     = one 27-base window of the suffix (layout in device_common.h):
//               bases zero-padded past the read end, then min(remaining, 27).
//               Comparing (bases, clamped length) is the order of Section 2
//               inside one window: a suffix that ends in the window is a
//               proper prefix of, hence below, one that goes on; equal keys
//               with a clamped length below 27 are identical suffixes, which
//               stable passes keep in read order.
//   * sort    = most-significant digit first.  Level 1 computes window-0 keys
//               from the 2-bit reads and scatters them by their top 8 bits
//               (keys are never stored unsorted); further 8-bit levels split
//               every bucket larger than one chunk (64 x 3, 6 or 8 suffixes,
//               the tuning's choice).  Runs of small buckets are then sorted
//               on their remaining digits, tie-refined window by window and
//               emitted by one wave, in LDS.  A tie on a full window (clamped
//               length 27) fetches the next window of the tied suffixes only,
//               one aligned 16-byte text record each.
//   * levels  = each level's scan hands on the next level's segment list and
//               its tile totals; the lists and their prefixes are built on the
//               device, so the host reads one small counter block per level,
//               and a build whose level kernels read their sizes on the
//               device can be captured whole in a hipGraph.
//
// Every pass is stable and the initial order is read-major, so suffixes that
// are equal through their terminators stay in read-index order (the stability
// argument of Section 3.2).

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "cxbwt.h"
#include "device_common.h"

namespace {

using namespace cxk;

// Tuning.  The level tile (suffixes per thread of a scatter) and the chunk
// (suffixes per lane of the one-wave chunk kernel) are template parameters;
// the library holds every listed instantiation and each build uses the one
// its thread selected (cxbwt_set_tuning).  Capacities are sized for the
// smallest tile and chunk, so a workspace fits every choice.
constexpr int LOCAL_WG = 64;                   // one wave finishes a chunk
constexpr int MIN_TILE_ITEMS = 6;
constexpr int MAX_TILE_ITEMS = 8;  // items per thread a histogram kernel loads at once
constexpr int MIN_CHUNK_ITEMS = 3;
constexpr int MIN_TILE = BLOCK * MIN_TILE_ITEMS;
constexpr int MIN_CHUNK = LOCAL_WG * MIN_CHUNK_ITEMS;
constexpr int GROUP_TILES = 256;               // tiles per first-stage scan group
constexpr uint64_t SEG_BATCH_MIN = 2048;       // segment size the level scratch is sized for

constexpr uint32_t ST_BAD_OFFSETS = 1u;
constexpr uint32_t ST_TOO_LONG = 2u;
constexpr uint32_t ST_BAD_CHAR = 4u;
constexpr uint32_t ST_LIST_OVERFLOW = 8u;
constexpr uint32_t ST_WINDOW_BOUND = 16u;
constexpr uint32_t ST_PLAN_MISMATCH = 32u;  // inputs no longer match a captured build

// counters block layout (uint32 slots; 64-bit values on even slots).  Chunk
// and big counts share one 64-bit word; the level kinds of the statistics
// block are folded into the 64-bit words from C_FOLD on; a build whose
// levels are scheduled on the device keeps its running totals (G_*) from
// C_CUM on.
enum { C_STATUS = 0, C_NFINAL = 1, C_NCHUNK = 2, C_NBIG = 3, C_NCUR = 4, C_FLAGS = 5, C_FOLD = 16, C_CUM = 32,
       C_COUNT = 64 };
enum { G_LEVELS, G_BIGSEG, G_LEVSUF, G_REGATH, G_MAXWIN, G_CHUNKS, G_FINALS, G_FINLEN, G_BATCHES, G_COUNT };
constexpr uint32_t FL_STALLED = 1u;     // a level did not fit the scratch: the host finishes the build
constexpr uint32_t FL_INCOMPLETE = 2u;  // segments remain after the last scheduled level

// A run of suffixes [start, start+len) in key/handle buffer `buf`, whose keys
// are for window r and agree on every digit before d.
// Positions fit 32 bits (at most CXBWT_MAX_BASES bases).
struct Seg {
  uint32_t start;
  uint32_t len;
  uint16_t r;
  uint8_t d;
  uint8_t buf : 1;
  uint8_t regather : 1;  // keys must be re-fetched for window r before use
  uint8_t unsplit : 1;   // chunk only: suffixes are in read order, not yet split by digit d
  uint32_t coll;         // collection the suffixes belong to
};
static_assert(sizeof(Seg) == 16, "segment records are 16 bytes");

// Where collection c's rows go.  Suffix position j (a base position of the
// whole batch) of collection c is BWT row j + row_shift of that collection,
// stored at output byte j + out_shift (the outputs of the collections are
// concatenated, each n_c + B_c bytes).
struct CollMap {
  uint64_t out_shift;  // reads in collections 0..c
  int64_t row_shift;   // n_c - (first base of c)
};

// Statistics counters are spread over STAT_SPREAD cache lines (indexed by
// workgroup) so that thousands of workgroups never queue on one address.
constexpr int STAT_SPREAD = 64;
constexpr int STAT_STRIDE = 16;  // u64 counters per 128-byte line
// Kinds: window fetches, scattered suffixes, then what a level's scan
// produced (folded and cleared after every scan): suffixes, re-keyed
// suffixes, largest window, tiles and scan groups of the next level's
// segments, and suffixes and tiles of the final groups.
enum {
  K_FETCHES = 0,
  K_SCATTERED,
  K_NEXT_LEN,
  K_NEXT_REGATHER,
  K_NEXT_MAXR,
  K_NEXT_TILES,
  K_NEXT_GROUPS,
  K_FINAL_LEN,
  K_FINAL_TILES,
  K_KINDS
};
constexpr int K_LEVEL_FIRST = K_NEXT_LEN;
constexpr int K_LEVEL_KINDS = K_KINDS - K_NEXT_LEN;
constexpr uint64_t STAT_KIND = (uint64_t)STAT_SPREAD * STAT_STRIDE;
constexpr uint64_t STAT_WORDS = K_KINDS * STAT_KIND;
__device__ __forceinline__ unsigned long long *stat_slot(unsigned long long *base) {
  return base + (blockIdx.x % STAT_SPREAD) * STAT_STRIDE;
}

struct Lists {
  Seg *big_next;
  uint32_t *n_big_next;          // high half of *n_chunk_big
  uint32_t cap_big;
  Seg *chunks;
  unsigned long long *n_chunk_big;  // chunk count (low 32 bits), big count (high)
  uint32_t cap_chunks;
  Seg *finals;
  uint32_t *n_finals;
  uint32_t cap_finals;
  uint32_t *status;
  uint32_t rmax;
  unsigned long long *stats;  // the statistics block (K_* kinds)
  uint32_t chunk;  // largest run finished by one wave (the selected chunk size)
  uint32_t tile_len;  // suffixes per level tile
};

// Number of read starts strictly before base p: for the first base of a
// read, the index of that read among the non-empty reads.  srank[w] counts
// the starts at positions below 16w.
__device__ __forceinline__ uint32_t start_rank(const TextRec *__restrict__ text, const uint32_t *__restrict__ srank,
                                               uint64_t p) {
  const uint64_t below = text[p >> 4].lo & ((1ull << (p & 15)) - 1ull);
  return srank[p >> 4] + (uint32_t)__popcll(below);
}

// Writes the BWT row of a sorted suffix; an offset-0 suffix also records its
// row under its read's rank among the non-empty reads (k_term turns those
// into term_pos).
__device__ __forceinline__ void emit_row(uint64_t j, const CollMap &cm, uint64_t key, uint32_t p,
                                         const TextRec *__restrict__ text, const uint32_t *__restrict__ srank,
                                         uint8_t *__restrict__ bwt, uint64_t *__restrict__ start_row) {
  const uint32_t pv = (uint32_t)key & 7u;
  const uint32_t lut = 'A' | ('C' << 8) | ('G' << 16) | ('T' << 24);
  bwt[j + cm.out_shift] = pv == 4 ? (uint8_t)'$' : (uint8_t)((lut >> (8 * pv)) & 0xFFu);
  if (pv == 4) start_row[start_rank(text, srank, p)] = (uint64_t)((int64_t)j + cm.row_shift);
}

// Base t of the packed input (2 bits, first base of a word highest).
__device__ __forceinline__ uint32_t base_at(const uint64_t *__restrict__ packed, uint64_t t) {
  return (uint32_t)(packed[t >> 5] >> (62 - 2 * (t & 31))) & 3u;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  The
// scatters give consecutive tiles to the same XCD (tile = xcd * (N/8) + k
// for the k-th workgroup of an XCD), so that the partial cache lines that
// neighbouring tiles write into one bucket meet in the same L2.
#ifndef CXBWT_XCDS
#define CXBWT_XCDS 8
#endif
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
  const uint32_t per = n / CXBWT_XCDS;
  const uint32_t full = per * CXBWT_XCDS;
  if (CXBWT_XCDS <= 1 || b >= full) return b;
  return (b % CXBWT_XCDS) * per + b / CXBWT_XCDS;
}

__device__ __forceinline__ uint32_t find_upper(const uint32_t *prefix, uint32_t count, uint32_t x) {
  // largest s < count with prefix[s] <= x (prefix[0] == 0, non-decreasing)
  uint32_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// a0: read packing (ASCII -> 2-bit, first base in the top bits)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t base_code(uint32_t c, bool &bad) {
  // A C G T = 0x41 0x43 0x47 0x54 -> 0 1 2 3 by bits 2..1 of c ^ (c >> 1)
  bad |= !(c == 'A' || c == 'C' || c == 'G' || c == 'T');
  return ((c >> 2) ^ (c >> 1)) & 3u;
}

// One thread per 32-base word.  Full words with a 16-byte aligned source
// are read as two 16-byte loads (a wave covers 2 KB contiguously); the tail
// word and unaligned sources go byte by byte.
__global__ void k_pack(const uint8_t *__restrict__ ascii, uint64_t nb, uint64_t *__restrict__ packed, uint64_t nwords,
                       uint32_t *status) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  const uint64_t t0 = w * 32;
  uint64_t x = 0;
  bool bad = false;
  if (t0 + 32 <= nb && ((uintptr_t)ascii & 15) == 0) {
    const uint4 *src = reinterpret_cast<const uint4 *>(ascii + t0);
    const uint4 a = src[0], b = src[1];
    const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = q * 4 + k;  // little-endian: byte k of word q is base j
        x |= (uint64_t)base_code((v[q] >> (8 * k)) & 0xFFu, bad) << (62 - 2 * j);
      }
    }
  } else {
    for (int j = 0; j < 32; ++j) {
      const uint64_t t = t0 + j;
      if (t >= nb) break;
      x |= (uint64_t)base_code(ascii[t], bad) << (62 - 2 * j);
    }
  }
  packed[w] = x;
  if (bad && status) atomicOr(status, ST_BAD_CHAR);
}

// ---------------------------------------------------------------------------
// read preparation: validate offsets, mark read starts in a bitmap (bit t of
// word t/32 for position t), emit the n rows of the bare terminators (row i =
// $_i, preceded by the last base of read i)
// ---------------------------------------------------------------------------
__global__ void k_prep(const uint64_t *__restrict__ packed, const uint64_t *__restrict__ offsets, uint64_t n, uint64_t nb,
                       uint32_t maxlen, const uint64_t *__restrict__ coll_reads, uint32_t ncoll,
                       uint32_t *sbits, uint8_t *__restrict__ bwt, uint64_t *__restrict__ term_pos,
                       uint32_t *status) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // collection of read i: largest c with coll_reads[c] <= i
  uint32_t clo = 0, chi = ncoll;
  while (chi - clo > 1) {
    const uint32_t mid = (clo + chi) >> 1;
    if (coll_reads[mid] <= i) clo = mid;
    else chi = mid;
  }
  const uint64_t first_read = coll_reads[clo];
  const uint64_t a = offsets[i], b = offsets[i + 1];
  const bool bad = b < a || b > nb || (i == 0 && a != 0) || (i == n - 1 && b != nb);
  if (bad) {
    atomicOr(status, ST_BAD_OFFSETS);
    return;
  }
  if (b - a > (uint64_t)maxlen) {
    atomicOr(status, ST_TOO_LONG);
    return;
  }
  // row (i - first_read) of the collection, whose output starts at byte
  // (bases before it) + (reads before it): byte offsets[first_read] + i.
  // Valid offsets never decrease, so the collection's first offset is at
  // most a; checking it keeps every write in bounds when another read's
  // offsets are the invalid ones.
  const uint64_t ob = offsets[first_read];
  if (ob > a) {
    atomicOr(status, ST_BAD_OFFSETS);
    return;
  }
  const uint64_t out = ob + i;
  if (i == n - 1) atomicOr(&sbits[nb >> 5], 1u << (nb & 31));  // end of the text
  if (b > a) {
    const uint64_t e = b - 1;
    atomicOr(&sbits[a >> 5], 1u << (a & 31));
    const uint32_t lut = 'A' | ('C' << 8) | ('G' << 16) | ('T' << 24);
    bwt[out] = (uint8_t)((lut >> (8 * base_at(packed, e))) & 0xFFu);
  } else {
    bwt[out] = (uint8_t)'$';
    term_pos[i] = i - first_read;
  }
}

// 32 bases of the packed input starting at position t (a multiple of 16),
// first base highest; words past the input read as zero.
__device__ __forceinline__ uint64_t packed_at16(const uint64_t *__restrict__ packed, uint64_t nwords, uint64_t t) {
  const uint64_t k = t >> 5;
  const uint64_t w0 = k < nwords ? packed[k] : 0ull;
  if (!(t & 31)) return w0;
  const uint64_t w1 = k + 1 < nwords ? packed[k + 1] : 0ull;
  return (w0 << 32) | (w1 >> 32);
}

// Text records from the packed bases and the read-start bitmap (k_prep);
// the bitmap holds at least floor(B/32) + 4 zero-padded words.
__global__ void k_text_records(const uint64_t *__restrict__ packed, uint64_t nwords, const uint32_t *__restrict__ sbits,
                               TextRec *__restrict__ text, uint64_t nrec) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nrec) return;
  const uint64_t t = 16 * w;
  TextRec r;
  r.hi = packed_at16(packed, nwords, t);
  const uint64_t tail = packed_at16(packed, nwords, t + 32) & ~((1ull << 44) - 1);  // bases t+32 .. t+41
  const uint64_t prev = w ? (packed_at16(packed, nwords, t - 16) >> 32) & 3ull : 0ull;  // base t-1
  const uint64_t k = t >> 5;
  const uint64_t bits = (((uint64_t)sbits[k + 1] << 32) | sbits[k]) >> (t & 31);
  r.lo = tail | (prev << 42) | (bits & REC_STARTS);
  text[w] = r;
}

// First base of every collection (host needs them to lay out segments).
__global__ void k_coll_bases(const uint64_t *__restrict__ offsets, const uint64_t *__restrict__ coll_reads,
                             uint32_t ncoll, uint64_t *__restrict__ bases) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= ncoll) bases[c] = offsets[coll_reads[c]];
}

// ---------------------------------------------------------------------------
// exclusive prefix counts of the read starts, per text record (each record
// owns the start bits of its first 16 positions)
// ---------------------------------------------------------------------------
constexpr int RANK_WPT = 16;                      // words per thread
constexpr int RANK_BLOCK_WORDS = BLOCK * RANK_WPT;

// Counted on the read-start bitmap (32 positions a word, two records).
__global__ __launch_bounds__(BLOCK) void k_rank_count(const uint32_t *__restrict__ sbits, uint64_t nw,
                                                      uint32_t *__restrict__ blocksum) {
  __shared__ uint32_t tmp[WAVES];
  const uint64_t w0 = (uint64_t)blockIdx.x * RANK_BLOCK_WORDS + (uint64_t)threadIdx.x * RANK_WPT;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < RANK_WPT; ++i)
    if (w0 + i < nw) c += (uint32_t)__popc(sbits[w0 + i]);
  uint32_t total;
  block_excl_sum(c, tmp, &total);
  if (threadIdx.x == 0) blocksum[blockIdx.x] = total;
}

__global__ __launch_bounds__(BLOCK) void k_rank_top(uint32_t *__restrict__ blocksum, uint32_t nblocks) {
  __shared__ uint32_t tmp[WAVES];
  uint32_t running = 0;
  for (uint32_t base = 0; base < nblocks; base += BLOCK) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < nblocks ? blocksum[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_excl_sum(v, tmp, &total);
    if (i < nblocks) blocksum[i] = running + ex;
    running += total;
  }
}

// srank of records 2k and 2k+1 from bitmap word k.
__global__ __launch_bounds__(BLOCK) void k_rank_words(const uint32_t *__restrict__ sbits, uint64_t nw,
                                                      const uint32_t *__restrict__ blocksum,
                                                      uint32_t *__restrict__ srank, uint64_t nrec) {
  __shared__ uint32_t tmp[WAVES];
  const uint64_t w0 = (uint64_t)blockIdx.x * RANK_BLOCK_WORDS + (uint64_t)threadIdx.x * RANK_WPT;
  uint32_t word[RANK_WPT];
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < RANK_WPT; ++i) {
    word[i] = w0 + i < nw ? sbits[w0 + i] : 0u;
    c += (uint32_t)__popc(word[i]);
  }
  uint32_t run = blocksum[blockIdx.x] + block_excl_sum(c, tmp, nullptr);
#pragma unroll
  for (int i = 0; i < RANK_WPT; ++i) {
    const uint64_t r0 = 2 * (w0 + i);
    if (r0 < nrec) srank[r0] = run;
    if (r0 + 1 < nrec) srank[r0 + 1] = run + (uint32_t)__popc(word[i] & 0xFFFFu);
    run += (uint32_t)__popc(word[i]);
  }
}

// term_pos of every non-empty read from the row its offset-0 suffix recorded.
// (A replayed graph runs this even when k_prep found the offsets invalid:
// reads that leave the text are skipped, and the result is then reported
// as an error.)
__global__ void k_term(const uint64_t *__restrict__ offsets, uint64_t n, uint64_t nb,
                       const TextRec *__restrict__ text, const uint32_t *__restrict__ srank,
                       const uint64_t *__restrict__ start_row, uint64_t *__restrict__ term_pos) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t a = offsets[i], b = offsets[i + 1];
  if (b > a && b <= nb) term_pos[i] = start_row[start_rank(text, srank, a)];
}

// ---------------------------------------------------------------------------
// a1 for collections that fit one chunk: window-0 keys in read order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(BLOCK) void k_gen(const Seg *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                                               uint32_t nsegs, uint32_t tile_len, const TextRec *__restrict__ text,
                                               uint64_t nb, uint64_t *__restrict__ keys, uint32_t *__restrict__ hdl) {
  const uint32_t tile = blockIdx.x;
  const uint32_t s = find_upper(tile_prefix, nsegs, tile);
  const Seg sg = segs[s];
  const uint64_t t0 = sg.start + (uint64_t)(tile - tile_prefix[s]) * tile_len;
  const uint64_t t1 = min(t0 + (uint64_t)tile_len, sg.start + sg.len);
  for (uint64_t p = t0 + threadIdx.x; p < t1; p += BLOCK) {
    keys[p] = first_key(text, nb, p);
    hdl[p] = (uint32_t)p;
  }
}

// ---------------------------------------------------------------------------
// a1 + a2, level 1: window-0 keys of every suffix of a collection (read
// order, from the 2-bit reads) counted by their top digit, then recomputed
// and scattered; keys are never stored unsorted.  One segment per collection.
// ---------------------------------------------------------------------------
template <int SUBT>
__global__ __launch_bounds__(BLOCK) void k_gen_hist(const Seg *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                                                    uint32_t nsegs, uint32_t tile_len, const TextRec *__restrict__ text,
                                                    uint64_t nb, uint32_t *__restrict__ tile_hist) {
  __shared__ uint32_t hist[256];
  const uint32_t tile = blockIdx.x;
  const uint32_t s = find_upper(tile_prefix, nsegs, tile);
  const Seg sg = segs[s];
  const uint64_t t0 = sg.start + (uint64_t)(tile - tile_prefix[s]) * tile_len;
  const uint64_t t1 = min(t0 + (uint64_t)tile_len, sg.start + sg.len);
  hist[threadIdx.x] = 0;
  __syncthreads();
  // every record load of a sub-tile is issued before its first count
#pragma unroll
  for (int sub = 0; sub < SUBT; ++sub) {
    const uint64_t u0 = t0 + (uint64_t)sub * BLOCK * MAX_TILE_ITEMS;
    uint64_t kk[MAX_TILE_ITEMS];
#pragma unroll
    for (int i = 0; i < MAX_TILE_ITEMS; ++i) {
      const uint64_t p = u0 + (uint64_t)i * BLOCK + threadIdx.x;
      if (p < t1) kk[i] = first_key(text, nb, p);
    }
#pragma unroll
    for (int i = 0; i < MAX_TILE_ITEMS; ++i)
      if (u0 + (uint64_t)i * BLOCK + threadIdx.x < t1) atomicAdd(&hist[digit_of(kk[i], 0)], 1u);
  }
  __syncthreads();
  tile_hist[(uint64_t)tile * 256 + threadIdx.x] = hist[threadIdx.x];
}

// Stable scatter of `m` items held in registers to global positions
// base[digit] + rank-within-tile, staged through LDS so that each digit's run
// is written contiguously.  A tile is NW waves x TI items: the wide tile
// (8 waves, 4096 suffixes) writes runs twice as long per bucket, which the
// memory system turns into fuller line writes.
template <int TI, int NW>
struct ScatterSmem {
  // the per-wave digit counters are dead once every rank is known, before
  // the first staged write: they share the key staging area
  static_assert(NW * 256 * 4 <= 64 * NW * TI * 8, "counters fit the key stage");
  union {
    uint64_t sk[64 * NW * TI];
    uint32_t wcount[NW * 256];
  };
  uint32_t sh[64 * NW * TI];
  uint32_t dstart[256];
  uint64_t goff[256];
  uint32_t tmp[NW];
};

template <int TI, int NW>
__device__ __forceinline__ void tile_scatter(ScatterSmem<TI, NW> &S, const uint64_t (&kr)[TI],
                                             const uint32_t (&hr)[TI], const uint32_t (&dig)[TI], uint32_t m, int d,
                                             uint64_t *__restrict__ Ko, uint32_t *__restrict__ Ho) {
  uint32_t pos[TI];
  block_multisplit<TI, NW>(dig, pos, S.wcount, S.dstart, S.tmp);
  __syncthreads();  // every wave has read its counters before the stage is written
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    if (dig[i] != NODIGIT) {
      S.sk[pos[i]] = kr[i];
      S.sh[pos[i]] = hr[i];
    }
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < m; q += 64 * NW) {
    const uint64_t k = S.sk[q];
    const uint32_t dd = digit_of(k, d);
    const uint64_t g = S.goff[dd] + (q - S.dstart[dd]);
    Ko[g] = k;
    Ho[g] = S.sh[q];
  }
}

template <int TI, int NW>
__global__ __launch_bounds__(64 * NW) void k_gen_scatter(const Seg *__restrict__ segs,
                                                       const uint32_t *__restrict__ tile_prefix,
                                                       const uint32_t *__restrict__ group_prefix, uint32_t nsegs,
                                                       const TextRec *__restrict__ text, uint64_t nb,
                                                       const uint32_t *__restrict__ tile_hist,
                                                       const uint32_t *__restrict__ gsum, uint64_t *__restrict__ Ko,
                                                       uint32_t *__restrict__ Ho) {
  constexpr uint32_t TL = 64 * NW * TI;
  __shared__ ScatterSmem<TI, NW> S;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint32_t s = find_upper(tile_prefix, nsegs, tile);
  const Seg sg = segs[s];
  const uint32_t tl = tile - tile_prefix[s];
  const uint64_t t0 = sg.start + (uint64_t)tl * TL;
  const uint32_t m = (uint32_t)min((uint64_t)TL, sg.start + sg.len - t0);
  uint64_t kr[TI];
  uint32_t hr[TI], dig[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const uint32_t li = item_index<TI>(i);
    if (li < m) {
      kr[i] = first_key(text, nb, t0 + li);
      hr[i] = (uint32_t)(t0 + li);
      dig[i] = digit_of(kr[i], 0);
    } else {
      kr[i] = 0;
      hr[i] = 0;
      dig[i] = NODIGIT;
    }
  }
  const uint32_t g = group_prefix[s] + tl / GROUP_TILES;
  if (threadIdx.x < 256)
    S.goff[threadIdx.x] =
        (uint64_t)gsum[(uint64_t)g * 256 + threadIdx.x] + tile_hist[(uint64_t)tile * 256 + threadIdx.x];
  tile_scatter(S, kr, hr, dig, m, 0, Ko, Ho);
}

// ---------------------------------------------------------------------------
// a2/a3 levels 2..: split every oversized segment by one 8-bit digit
// ---------------------------------------------------------------------------

// Per-tile digit histogram and per-segment OR/AND of the ordering bits.  A
// segment flagged `regather` first re-fetches its keys for window r.
//
// Kernels of levels 2.. take their segment count from dev_nsegs when it is
// given (a launch whose size was fixed before the count was known) and loop
// over their work with the grid's stride; with the count passed by value
// the grid covers the work and each workgroup takes one item.
template <bool PERSIST, int SUBT>
__global__ __launch_bounds__(BLOCK) void k_level_hist(const Seg *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                                                      uint32_t nsegs, const uint32_t *__restrict__ dev_nsegs,
                                                      uint32_t tile_len, uint64_t *keys0,
                                                      uint64_t *keys1, const uint32_t *__restrict__ hdl0,
                                                      const uint32_t *__restrict__ hdl1,
                                                      const TextRec *__restrict__ text, uint64_t nb,
                                                      uint32_t *__restrict__ tile_hist, unsigned long long *seg_or,
                                                      unsigned long long *seg_and) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t red[WAVES];
  if (dev_nsegs) nsegs = *dev_nsegs;
  if (nsegs == 0) return;
  const uint32_t ntiles = PERSIST ? tile_prefix[nsegs] : blockIdx.x + 1;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
  const uint32_t s = find_upper(tile_prefix, nsegs, tile);
  const Seg sg = segs[s];
  const uint64_t t0 = sg.start + (uint64_t)(tile - tile_prefix[s]) * tile_len;
  const uint64_t t1 = min(t0 + (uint64_t)tile_len, sg.start + sg.len);
  uint64_t *K = sg.buf ? keys1 : keys0;
  const uint32_t *H = sg.buf ? hdl1 : hdl0;
  hist[threadIdx.x] = 0;
  __syncthreads();
  // all loads of a sub-tile (keys, and for a re-keyed segment handles and
  // then records) are issued before any result is used
  uint64_t o = 0, a = ~0ull;
  // SUBT sub-tiles of BLOCK * MAX_TILE_ITEMS (two for the wide tile)
#pragma unroll
  for (int sub = 0; sub < SUBT; ++sub) {
    const uint64_t u0 = t0 + (uint64_t)sub * BLOCK * MAX_TILE_ITEMS;
    uint64_t kk[MAX_TILE_ITEMS];
    bool in[MAX_TILE_ITEMS];
#pragma unroll
    for (int i = 0; i < MAX_TILE_ITEMS; ++i) {
      const uint64_t j = u0 + (uint64_t)i * BLOCK + threadIdx.x;
      in[i] = j < t1;
      if (in[i]) kk[i] = K[j];
    }
    if (sg.regather) {
      uint32_t hh[MAX_TILE_ITEMS];
      TextRec tr[MAX_TILE_ITEMS];
#pragma unroll
      for (int i = 0; i < MAX_TILE_ITEMS; ++i)
        if (in[i]) hh[i] = H[u0 + (uint64_t)i * BLOCK + threadIdx.x];
#pragma unroll
      for (int i = 0; i < MAX_TILE_ITEMS; ++i)
        if (in[i]) tr[i] = window_load(text, nb, hh[i], sg.r);
#pragma unroll
      for (int i = 0; i < MAX_TILE_ITEMS; ++i)
        if (in[i]) {
          kk[i] = window_combine(tr[i], nb, hh[i], sg.r, (uint32_t)kk[i] & 7u);
          K[u0 + (uint64_t)i * BLOCK + threadIdx.x] = kk[i];
        }
    }
#pragma unroll
    for (int i = 0; i < MAX_TILE_ITEMS; ++i)
      if (in[i]) {
        atomicAdd(&hist[digit_of(kk[i], sg.d)], 1u);
        o |= kk[i];
        a &= kk[i];
      }
  }
  o = block_or(o, red);
  a = block_and(a, red);
  if (threadIdx.x == 0) {
    atomicOr(&seg_or[s], (unsigned long long)order_bits(o));
    atomicAnd(&seg_and[s], (unsigned long long)(a | 7ull));
  }
  tile_hist[(uint64_t)tile * 256 + threadIdx.x] = hist[threadIdx.x];
  if (!PERSIST) break;
  }
}

// First scan stage: inside each group of at most GROUP_TILES consecutive
// tiles of one segment, turn tile counts into exclusive prefixes per digit
// and record the group totals.  Sixteen tile counts are loaded before any
// is rewritten, so the loop waits for memory once per sixteen tiles.
template <bool PERSIST>
__global__ __launch_bounds__(BLOCK) void k_group_scan(const uint32_t *__restrict__ tile_prefix,
                                                      const uint32_t *__restrict__ group_prefix, uint32_t nsegs,
                                                      const uint32_t *__restrict__ dev_nsegs,
                                                      uint32_t *__restrict__ tile_hist, uint32_t *__restrict__ gsum) {
  constexpr uint32_t NB = 16;
  if (dev_nsegs) nsegs = *dev_nsegs;
  if (nsegs == 0) return;
  const uint32_t ngroups = PERSIST ? group_prefix[nsegs] : blockIdx.x + 1;
  for (uint32_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
  const uint32_t s = find_upper(group_prefix, nsegs, g);
  const uint32_t tb = tile_prefix[s] + (g - group_prefix[s]) * GROUP_TILES;
  const uint32_t te = min(tb + (uint32_t)GROUP_TILES, tile_prefix[s + 1]);
  const uint32_t d = threadIdx.x;
  uint32_t run = 0;
  uint32_t t = tb;
  for (; t + NB <= te; t += NB) {
    uint32_t x[NB];
#pragma unroll
    for (uint32_t j = 0; j < NB; ++j) x[j] = tile_hist[(uint64_t)(t + j) * 256 + d];
#pragma unroll
    for (uint32_t j = 0; j < NB; ++j) {
      tile_hist[(uint64_t)(t + j) * 256 + d] = run;
      run += x[j];
    }
  }
  for (; t < te; ++t) {
    const uint64_t at = (uint64_t)t * 256 + d;
    const uint32_t c = tile_hist[at];
    tile_hist[at] = run;
    run += c;
  }
  gsum[(uint64_t)g * 256 + d] = run;
  if (!PERSIST) break;
  }
}

// Digit totals of groups [g0, g1) added into cv (digit i*64 + lane in slot
// i), eight groups in flight.
__device__ __forceinline__ void group_totals(const uint32_t *__restrict__ gsum, uint32_t g0, uint32_t g1,
                                             uint32_t (&cv)[4]) {
  const uint32_t l = lane_id();
  uint32_t g = g0;
  for (; g + 8 <= g1; g += 8) {
    uint32_t x[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) x[j][i] = gsum[(uint64_t)(g + j) * 256 + i * 64 + l];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) cv[i] += x[j][i];
  }
  for (; g < g1; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) cv[i] += gsum[(uint64_t)g * 256 + i * 64 + l];
}

// Group totals of groups [g0, g1) replaced by the running bucket positions
// (starting at run), eight groups in flight.
__device__ __forceinline__ void group_starts(uint32_t *__restrict__ gsum, uint32_t g0, uint32_t g1,
                                             uint32_t (&run)[4]) {
  const uint32_t l = lane_id();
  uint32_t g = g0;
  for (; g + 8 <= g1; g += 8) {
    uint32_t x[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) x[j][i] = gsum[(uint64_t)(g + j) * 256 + i * 64 + l];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gsum[(uint64_t)(g + j) * 256 + i * 64 + l] = run[i];
        run[i] += x[j][i];
      }
  }
  for (; g < g1; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t at = (uint64_t)g * 256 + i * 64 + l;
      const uint32_t c = gsum[at];
      gsum[at] = run[i];
      run[i] += c;
    }
}

// First set bit at or above `from` of a 256-bit mask held as four words;
// 256 when there is none.
__device__ __forceinline__ uint32_t first_set_from(const uint64_t (&m)[4], uint32_t from) {
  uint32_t res = 256;
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    uint64_t x = m[i];
    if (from >= (uint32_t)(i + 1) * 64) x = 0;
    else if (from > (uint32_t)i * 64) x &= ~0ull << (from - (uint32_t)i * 64);
    if (x) res = (uint32_t)i * 64 + (uint32_t)__builtin_ctzll(x);
  }
  return res;
}

// Value of bucket b (< 256) of a wave-distributed 256-entry array (bucket
// i*64 + lane in slot i), the same in every lane.
__device__ __forceinline__ uint32_t bucket_at(const uint32_t (&v)[4], uint32_t b) {
  const int ln = (int)(b & 63);
  const uint32_t x0 = (uint32_t)__builtin_amdgcn_readlane((int)v[0], ln);
  const uint32_t x1 = (uint32_t)__builtin_amdgcn_readlane((int)v[1], ln);
  const uint32_t x2 = (uint32_t)__builtin_amdgcn_readlane((int)v[2], ln);
  const uint32_t x3 = (uint32_t)__builtin_amdgcn_readlane((int)v[3], ln);
  const uint32_t i = b >> 6;
  return i == 0 ? x0 : i == 1 ? x1 : i == 2 ? x2 : x3;
}

// Sum over the wave, in every lane.
__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t bits_below_lane(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Second scan stage.  Each segment gets its digit totals from the group
// totals, its bucket starts and the start of every (group, digit) run, and
// its buckets are sorted into chunks (runs of consecutive small buckets of
// at most L.chunk suffixes), segments for the next level (buckets above
// L.chunk) and final groups of identical suffixes (an ended tie at the last
// digit).  A segment whose current digit is constant is not scattered: it
// moves to its first varying digit, or, when all its ordering bits agree, to
// the next window (a full tie) or to the final list (an ended tie).
//
// COOP = false: one wave per segment, WAVES segments per workgroup.
// COOP = true: one segment per workgroup, its groups shared by the waves
// (for segments spanning many groups).  All control below is uniform per
// wave: chunk boundaries come from a walk of one step per chunk over bucket
// masks, and the list entries are written by all lanes at once from
// positions reserved with one atomic per list per workgroup.
template <bool COOP, bool PERSIST>
__global__ __launch_bounds__(BLOCK) void k_level_scan(const Seg *__restrict__ segs,
                                                      const uint32_t *__restrict__ group_prefix, uint32_t nsegs,
                                                      uint32_t *__restrict__ gsum,
                                                      const unsigned long long *__restrict__ seg_or,
                                                      const unsigned long long *__restrict__ seg_and,
                                                      uint8_t *__restrict__ seg_split, Lists L, int force_split,
                                                      const uint32_t *__restrict__ dev_nsegs) {
  constexpr int CW = COOP ? 1 : WAVES;  // waves that classify a segment
  __shared__ uint32_t part[COOP ? WAVES : 1][256];
  __shared__ uint32_t cstart[CW][256];
  __shared__ uint32_t clen[CW][256];
  __shared__ uint32_t wbv[CW][257];  // bucket starts of the classifying wave, then the segment length
  __shared__ uint32_t wnx[CW][256];  // per bucket: end of a chunk starting there | next chunk start << 16
  __shared__ uint32_t wcnt[WAVES][3];
  __shared__ uint32_t wbase[WAVES][3];
  __shared__ uint32_t wstat[WAVES][K_LEVEL_KINDS];
  const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const uint32_t l = lane_id();
  if (dev_nsegs) nsegs = *dev_nsegs;
  constexpr uint32_t SPB = COOP ? 1u : (uint32_t)WAVES;  // segments per workgroup step
  for (uint32_t blk = blockIdx.x; blk * SPB < nsegs; blk += gridDim.x) {
  if (PERSIST) __syncthreads();  // the previous step's LDS reads are done
  const uint32_t s = COOP ? blk : blk * WAVES + w;
  const uint32_t cw = COOP ? 0 : w;  // this wave's chunk-list slot
  uint32_t cv[4] = {0, 0, 0, 0}, bv[4] = {0, 0, 0, 0};
  int mode = 0;  // 0: no segment, 1: passes through unsplit, 2: split by digit d
  Seg sg{};
  Seg nx{};
  int nx_list = 0;  // mode 1: 0 none, 1 next level, 2 final
  if (s < nsegs) {
    sg = segs[s];
    const uint32_t gp0 = group_prefix[s], gp1 = group_prefix[s + 1];
    uint32_t pre[4] = {0, 0, 0, 0};
    uint32_t ga = gp0, gb = gp1;
    if (COOP) {
      const uint32_t per = (gp1 - gp0 + WAVES - 1) / WAVES;
      ga = min(gp0 + w * per, gp1);
      gb = min(ga + per, gp1);
      uint32_t pc[4] = {0, 0, 0, 0};
      group_totals(gsum, ga, gb, pc);
#pragma unroll
      for (int i = 0; i < 4; ++i) part[w][i * 64 + l] = pc[i];
      __syncthreads();
      for (uint32_t ww = 0; ww < (uint32_t)WAVES; ++ww)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t x = part[ww][i * 64 + l];
          cv[i] += x;
          if (ww < w) pre[i] += x;
        }
    } else {
      group_totals(gsum, gp0, gp1, cv);
    }
    bool one = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) one |= cv[i] == sg.len;
    if (__ballot(one) && !force_split) {
      mode = 1;
      const unsigned long long o = seg_or[s], a = seg_and[s];
      const uint64_t diff = (o ^ a) & ~7ull;
      nx = sg;
      nx.regather = 0;
      if (diff == 0) {
        if (clamp_of(a) < (uint32_t)W) {
          nx = sg;
          nx_list = 2;
        } else if (sg.r + 1 > L.rmax) {
          if (l == 0 && (!COOP || w == 0)) atomicOr(L.status, ST_WINDOW_BOUND);
        } else {
          nx.r = sg.r + 1;
          nx.d = 0;
          nx.regather = 1;
          nx_list = 1;
        }
      } else {
        const int top = 63 - __builtin_clzll(diff);
        nx.d = (uint8_t)(top >= 8 ? (63 - top) >> 3 : 7);
        nx_list = 1;
      }
    } else {
      mode = 2;
      // bucket starts: exclusive scan over the digits in order
      uint32_t carry = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t inc = wave_incl_sum(cv[i]);
        bv[i] = carry + inc - cv[i];
        carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
      }
      uint32_t run[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) run[i] = sg.start + bv[i] + pre[i];
      group_starts(gsum, ga, gb, run);
    }
  }
  if (COOP && w != 0) mode = 0;  // wave 0 classifies the workgroup's segment

  uint32_t nc = 0, nbg = 0, nf = 0;
  uint64_t NB[4] = {0, 0, 0, 0}, FIN[4] = {0, 0, 0, 0};
  // what this wave hands on: K_NEXT_LEN .. K_FINAL_TILES
  uint32_t ls[K_LEVEL_KINDS] = {0, 0, 0, 0, 0, 0, 0};
  const uint32_t T = L.tile_len;
  if (mode == 1) {
    nbg = nx_list == 1;
    nf = nx_list == 2;
    const uint32_t nt = (nx.len + T - 1) / T;
    if (nx_list == 1) {
      ls[K_NEXT_LEN - K_LEVEL_FIRST] = nx.len;
      ls[K_NEXT_REGATHER - K_LEVEL_FIRST] = nx.regather ? nx.len : 0u;
      ls[K_NEXT_MAXR - K_LEVEL_FIRST] = nx.r;
      ls[K_NEXT_TILES - K_LEVEL_FIRST] = nt;
      ls[K_NEXT_GROUPS - K_LEVEL_FIRST] = (nt + GROUP_TILES - 1) / GROUP_TILES;
    } else if (nx_list == 2) {
      ls[K_FINAL_LEN - K_LEVEL_FIRST] = nx.len;
      ls[K_FINAL_TILES - K_LEVEL_FIRST] = nt;
    }
  } else if (mode == 2) {
    const uint32_t C = L.chunk;
    uint64_t NZS[4], BIG[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      NZS[i] = __ballot(cv[i] != 0 && cv[i] <= C);
      BIG[i] = __ballot(cv[i] > C);
    }
    // chunks: a chunk starts at a non-empty small bucket and takes the
    // following buckets while its size stays within C and no big bucket
    // intervenes.  Every lane first finds, for its four buckets b, where a
    // chunk starting at b would end (e: the first big bucket after b, or the
    // first bucket that would take the size above C, by binary search on the
    // bucket starts) and where the next chunk would start (the first
    // non-empty small bucket at or after e); the walk over the chunk starts
    // is then one LDS read per chunk.
#pragma unroll
    for (int i = 0; i < 4; ++i) wbv[cw][i * 64 + l] = bv[i];
    if (l == 0) wbv[cw][256] = sg.len;
    uint32_t big_after[4], nzs_after[4];  // first set bit in the words above word i
    {
      uint32_t fb = 256, fn = 256;
#pragma unroll
      for (int i = 3; i >= 0; --i) {
        big_after[i] = fb;
        nzs_after[i] = fn;
        if (BIG[i]) fb = (uint32_t)i * 64 + (uint32_t)__builtin_ctzll(BIG[i]);
        if (NZS[i]) fn = (uint32_t)i * 64 + (uint32_t)__builtin_ctzll(NZS[i]);
      }
    }
    const uint64_t above = ~(lanemask_lt() | (1ull << l));  // lanes above this one
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t b = (uint32_t)i * 64 + l;
      const uint32_t sb = bv[i];
      // largest x >= b whose prefix bv[x] + cv[x] = wbv[x + 1] stays within
      // sb + C (monotone in x); differences, so sb + C cannot wrap
      uint32_t x = b;
#pragma unroll
      for (uint32_t step = 128; step > 0; step >>= 1) {
        const uint32_t y = x + step;
        if (y < 256 && wbv[cw][y + 1] - sb <= C) x = y;
      }
      const uint64_t mb = BIG[i] & above;
      const uint32_t nbig = mb ? (uint32_t)i * 64 + (uint32_t)__builtin_ctzll(mb) : big_after[i];
      const uint32_t e = min(x + 1, nbig);
      uint32_t nxt = 256;
      if (e < 256) {
        const uint32_t w = e >> 6;
        const uint64_t word = w == 0 ? NZS[0] : w == 1 ? NZS[1] : w == 2 ? NZS[2] : NZS[3];
        const uint64_t m = word & (~0ull << (e & 63));
        const uint32_t after = w == 0 ? nzs_after[0] : w == 1 ? nzs_after[1] : w == 2 ? nzs_after[2] : nzs_after[3];
        nxt = m ? w * 64 + (uint32_t)__builtin_ctzll(m) : after;
      }
      wnx[cw][b] = e | (nxt << 16);
    }
    uint32_t b = first_set_from(NZS, 0);
    while (b < 256) {
      const uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane((int)wnx[cw][b]);
      const uint32_t e = v & 0xFFFFu;
      const uint32_t sb = (uint32_t)__builtin_amdgcn_readfirstlane((int)wbv[cw][b]);
      const uint32_t se = (uint32_t)__builtin_amdgcn_readfirstlane((int)wbv[cw][e]);
      if (l == 0) {
        cstart[cw][nc] = sb;
        clen[cw][nc] = se - sb;
      }
      ++nc;
      b = v >> 16;
    }
    if (sg.d == 7) {
      // bucket value b is the clamped length; all ordering bits agree
      FIN[0] = BIG[0] & ((1ull << W) - 1);
      NB[0] = BIG[0] & ~FIN[0];
      NB[1] = BIG[1];
      NB[2] = BIG[2];
      NB[3] = BIG[3];
      if ((NB[0] | NB[1] | NB[2] | NB[3]) && sg.r + 1 > L.rmax) {
        if (l == 0) atomicOr(L.status, ST_WINDOW_BOUND);
        NB[0] = NB[1] = NB[2] = NB[3] = 0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) NB[i] = BIG[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      nbg += (uint32_t)__popcll(NB[i]);
      nf += (uint32_t)__popcll(FIN[i]);
    }
    uint32_t blen = 0, btiles = 0, bgroups = 0, flen = 0, ftiles = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t nt = (cv[i] + T - 1) / T;
      if ((NB[i] >> l) & 1) {
        blen += cv[i];
        btiles += nt;
        bgroups += (nt + GROUP_TILES - 1) / GROUP_TILES;
      }
      if ((FIN[i] >> l) & 1) {
        flen += cv[i];
        ftiles += nt;
      }
    }
    blen = wave_total(blen);
    ls[K_NEXT_LEN - K_LEVEL_FIRST] = blen;
    ls[K_NEXT_REGATHER - K_LEVEL_FIRST] = sg.d == 7 ? blen : 0u;
    ls[K_NEXT_MAXR - K_LEVEL_FIRST] = nbg ? sg.r + (sg.d == 7 ? 1u : 0u) : 0u;
    ls[K_NEXT_TILES - K_LEVEL_FIRST] = wave_total(btiles);
    ls[K_NEXT_GROUPS - K_LEVEL_FIRST] = wave_total(bgroups);
    ls[K_FINAL_LEN - K_LEVEL_FIRST] = wave_total(flen);
    ls[K_FINAL_TILES - K_LEVEL_FIRST] = wave_total(ftiles);
    if (l == 0) {
      seg_split[s] = 1;
      atomicAdd(stat_slot(L.stats + K_SCATTERED * STAT_KIND), (unsigned long long)sg.len);
    }
  }
  if (mode == 1 && l == 0) seg_split[s] = 0;
  if (l == 0) {
    wcnt[w][0] = nc;
    wcnt[w][1] = nbg;
    wcnt[w][2] = nf;
#pragma unroll
    for (int k = 0; k < K_LEVEL_KINDS; ++k) wstat[w][k] = ls[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K_LEVEL_KINDS; ++k) {
      unsigned long long v = 0;
      for (int ww = 0; ww < WAVES; ++ww)
        v = (k + K_LEVEL_FIRST == K_NEXT_MAXR) ? max(v, (unsigned long long)wstat[ww][k]) : v + wstat[ww][k];
      unsigned long long *slot = stat_slot(L.stats + (k + K_LEVEL_FIRST) * STAT_KIND);
      if (v) {
        if (k + K_LEVEL_FIRST == K_NEXT_MAXR) atomicMax(slot, v);
        else atomicAdd(slot, v);
      }
    }
    uint32_t tc = 0, tb = 0, tf = 0;
    for (int ww = 0; ww < WAVES; ++ww) {
      wbase[ww][0] = tc;
      wbase[ww][1] = tb;
      wbase[ww][2] = tf;
      tc += wcnt[ww][0];
      tb += wcnt[ww][1];
      tf += wcnt[ww][2];
    }
    // one atomic reserves the chunk and big-segment slots together
    unsigned long long old = 0;
    if (tc || tb) old = atomicAdd(L.n_chunk_big, (unsigned long long)tc | ((unsigned long long)tb << 32));
    const uint32_t bf = tf ? atomicAdd(L.n_finals, tf) : 0u;
    for (int ww = 0; ww < WAVES; ++ww) {
      wbase[ww][0] += (uint32_t)old;
      wbase[ww][1] += (uint32_t)(old >> 32);
      wbase[ww][2] += bf;
    }
  }
  __syncthreads();
  const uint32_t base_c = wbase[w][0], base_b = wbase[w][1], base_f = wbase[w][2];
  bool overflow = false;
  if (mode == 1) {
    if (l == 0 && nx_list == 1) {
      if (base_b < L.cap_big) L.big_next[base_b] = nx;
      else overflow = true;
    }
    if (l == 0 && nx_list == 2) {
      if (base_f < L.cap_finals) L.finals[base_f] = nx;
      else overflow = true;
    }
  } else if (mode == 2) {
    const uint8_t nbuf = (uint8_t)(sg.buf ^ 1);
    for (uint32_t j = l; j < nc; j += 64) {
      const uint32_t at = base_c + j;
      if (at < L.cap_chunks) L.chunks[at] = Seg{sg.start + cstart[cw][j], clen[cw][j], sg.r, sg.d, nbuf, 0, 0, sg.coll};
      else overflow = true;
    }
    const bool last = sg.d == 7;
    uint32_t pb = 0, pf = 0;  // entries of the lower slots
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t st = sg.start + bv[i];
      if ((NB[i] >> l) & 1) {
        const uint32_t at = base_b + pb + bits_below_lane(NB[i]);
        const Seg e = last ? Seg{st, cv[i], (uint16_t)(sg.r + 1), 0, nbuf, 1, 0, sg.coll}
                           : Seg{st, cv[i], sg.r, (uint8_t)(sg.d + 1), nbuf, 0, 0, sg.coll};
        if (at < L.cap_big) L.big_next[at] = e;
        else overflow = true;
      }
      if ((FIN[i] >> l) & 1) {
        const uint32_t at = base_f + pf + bits_below_lane(FIN[i]);
        if (at < L.cap_finals) L.finals[at] = Seg{st, cv[i], sg.r, (uint8_t)(sg.d + 1), nbuf, 0, 0, sg.coll};
        else overflow = true;
      }
      pb += (uint32_t)__popcll(NB[i]);
      pf += (uint32_t)__popcll(FIN[i]);
    }
  }
  if (overflow) atomicOr(L.status, ST_LIST_OVERFLOW);
  if (!PERSIST) break;
  }
}

// Folds the level kinds of the statistics block into out[0..K_LEVEL_KINDS)
// (sums, a maximum for the window) and clears them for the next scan.  One
// wave.
__global__ __launch_bounds__(64) void k_level_fold(unsigned long long *__restrict__ stats,
                                                   unsigned long long *__restrict__ out,
                                                   const uint32_t *__restrict__ flags) {
  const uint32_t l = lane_id();
  if (flags && (*flags & (FL_STALLED | FL_INCOMPLETE))) return;  // keep what the host resumes from
  for (int k = K_LEVEL_FIRST; k < K_KINDS; ++k) {
    unsigned long long *slot = stats + k * STAT_KIND + (uint64_t)l * STAT_STRIDE;
    unsigned long long v = *slot;
    *slot = 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long t = __shfl_xor(v, o, 64);
      v = k == K_NEXT_MAXR ? max(v, t) : v + t;
    }
    if (l == 0) out[k - K_LEVEL_FIRST] = v;
  }
}

// Clears the per-segment OR/AND words of the segments counted at *dev_n.
__global__ void k_fill_seg(unsigned long long *__restrict__ seg_or, unsigned long long *__restrict__ seg_and,
                           const uint32_t *__restrict__ dev_n) {
  const uint32_t n = *dev_n;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    seg_or[i] = 0;
    seg_and[i] = ~0ull;
  }
}

// Between two levels of a build scheduled on the device (one thread): adds
// the finished level's chunks and final groups to the running totals, then
// makes the segments the level handed on the current ones (C_NCUR), or
// flags the build for the host when they would not fit the scratch or when
// no level is left.
__global__ void k_level_step(uint32_t *__restrict__ c, uint64_t seg_slots, uint64_t max_tiles, uint64_t max_groups,
                             int last) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t fl = c[C_FLAGS];
  if (fl & (FL_STALLED | FL_INCOMPLETE)) return;
  const unsigned long long *f = reinterpret_cast<const unsigned long long *>(c + C_FOLD);
  unsigned long long *g = reinterpret_cast<unsigned long long *>(c + C_CUM);
  g[G_CHUNKS] += c[C_NCHUNK];
  g[G_FINALS] += c[C_NFINAL];
  g[G_FINLEN] += f[K_FINAL_LEN - K_LEVEL_FIRST];
  c[C_NCHUNK] = 0;
  c[C_NFINAL] = 0;
  c[C_NCUR] = 0;
  const uint32_t nbig = c[C_NBIG];
  if (nbig == 0) return;
  if (last) {
    c[C_FLAGS] = fl | FL_INCOMPLETE;
    return;
  }
  if (nbig > seg_slots || f[K_NEXT_TILES - K_LEVEL_FIRST] > max_tiles ||
      f[K_NEXT_GROUPS - K_LEVEL_FIRST] > max_groups) {
    c[C_FLAGS] = fl | FL_STALLED;
    return;
  }
  c[C_NCUR] = nbig;
  c[C_NBIG] = 0;
  g[G_LEVELS] += 1;
  g[G_BIGSEG] += nbig;
  g[G_LEVSUF] += f[K_NEXT_LEN - K_LEVEL_FIRST];
  g[G_REGATH] += f[K_NEXT_REGATHER - K_LEVEL_FIRST];
  g[G_MAXWIN] = max(g[G_MAXWIN], f[K_NEXT_MAXR - K_LEVEL_FIRST]);
  g[G_BATCHES] += 1;
}

// A replayed build checks that the collection bases are those it was
// captured for.
__global__ void k_check_bases(const uint64_t *__restrict__ got, const uint64_t *__restrict__ want, uint32_t count,
                              uint32_t *status) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && got[i] != want[i]) atomicOr(status, ST_PLAN_MISMATCH);
}

// Tile and group prefixes of a segment list on the device.  Entries sit
// item_index<SEGP_ITEMS> in each workgroup of BLOCK threads; k_seg_count
// writes per-workgroup totals (tiles, groups), k_seg_scan adds the totals
// of the workgroups before it, writes tile_prefix[i] and group_prefix[i]
// (and entry n: the totals) and, when copy is given, the list itself.
constexpr int SEGP_ITEMS = 16;
constexpr uint32_t SEGP_WG = BLOCK * SEGP_ITEMS;

__device__ __forceinline__ void seg_tiles(const Seg *__restrict__ list, uint32_t n, uint32_t tile_len,
                                          uint32_t (&t)[SEGP_ITEMS], uint32_t (&g)[SEGP_ITEMS]) {
#pragma unroll
  for (int i = 0; i < SEGP_ITEMS; ++i) {
    const uint64_t at = (uint64_t)blockIdx.x * SEGP_WG + item_index<SEGP_ITEMS>(i);
    const uint32_t len = at < n ? list[at].len : 0u;
    t[i] = (len + tile_len - 1) / tile_len;
    g[i] = (t[i] + GROUP_TILES - 1) / GROUP_TILES;
  }
}

__global__ __launch_bounds__(BLOCK) void k_seg_count(const Seg *__restrict__ list, uint32_t n,
                                                     const uint32_t *__restrict__ dev_n, uint32_t tile_len,
                                                     uint32_t *__restrict__ wg_tot) {
  __shared__ uint32_t tmp[WAVES];
  if (dev_n) n = *dev_n;
  if ((uint64_t)blockIdx.x * SEGP_WG >= n) return;
  uint32_t t[SEGP_ITEMS], g[SEGP_ITEMS];
  seg_tiles(list, n, tile_len, t, g);
  uint32_t st = 0, sgr = 0;
#pragma unroll
  for (int i = 0; i < SEGP_ITEMS; ++i) {
    st += t[i];
    sgr += g[i];
  }
  uint32_t tt = 0, tg = 0;
  (void)block_excl_sum(st, tmp, &tt);
  (void)block_excl_sum(sgr, tmp, &tg);
  if (threadIdx.x == 0) {
    wg_tot[2 * blockIdx.x] = tt;
    wg_tot[2 * blockIdx.x + 1] = tg;
  }
}

__global__ __launch_bounds__(BLOCK) void k_seg_scan(const Seg *__restrict__ list, uint32_t n,
                                                    const uint32_t *__restrict__ dev_n, uint32_t tile_len,
                                                    const uint32_t *__restrict__ wg_tot, Seg *__restrict__ copy,
                                                    uint32_t *__restrict__ tile_prefix,
                                                    uint32_t *__restrict__ group_prefix) {
  __shared__ uint32_t tmp[WAVES];
  __shared__ uint32_t wt[WAVES][2];
  if (dev_n) n = *dev_n;
  if ((uint64_t)blockIdx.x * SEGP_WG >= n) return;
  // base of this workgroup: the totals of the workgroups before it
  uint32_t bt = 0, bg = 0;
  for (uint32_t k = threadIdx.x; k < blockIdx.x; k += BLOCK) {
    bt += wg_tot[2 * k];
    bg += wg_tot[2 * k + 1];
  }
  uint32_t sum_t = 0, sum_g = 0;
  (void)block_excl_sum(bt, tmp, &sum_t);
  (void)block_excl_sum(bg, tmp, &sum_g);
  uint32_t t[SEGP_ITEMS], g[SEGP_ITEMS];
  seg_tiles(list, n, tile_len, t, g);
  // exclusive prefixes inside the wave, items in item_index order
  const uint32_t w = threadIdx.x >> 6;
  uint32_t pt[SEGP_ITEMS], pg[SEGP_ITEMS];
  uint32_t ct = 0, cg = 0;
#pragma unroll
  for (int i = 0; i < SEGP_ITEMS; ++i) {
    const uint32_t it = wave_incl_sum(t[i]), ig = wave_incl_sum(g[i]);
    pt[i] = ct + it - t[i];
    pg[i] = cg + ig - g[i];
    ct += (uint32_t)__builtin_amdgcn_readlane((int)it, 63);
    cg += (uint32_t)__builtin_amdgcn_readlane((int)ig, 63);
  }
  if (lane_id() == 0) {
    wt[w][0] = ct;
    wt[w][1] = cg;
  }
  __syncthreads();
  uint32_t wbt = sum_t, wbg = sum_g;
  for (uint32_t ww = 0; ww < w; ++ww) {
    wbt += wt[ww][0];
    wbg += wt[ww][1];
  }
#pragma unroll
  for (int i = 0; i < SEGP_ITEMS; ++i) {
    const uint64_t at = (uint64_t)blockIdx.x * SEGP_WG + item_index<SEGP_ITEMS>(i);
    if (at < n) {
      tile_prefix[at] = wbt + pt[i];
      if (group_prefix) group_prefix[at] = wbg + pg[i];
      if (copy) copy[at] = list[at];
      if (at == n - 1) {
        tile_prefix[n] = wbt + pt[i] + t[i];
        if (group_prefix) group_prefix[n] = wbg + pg[i] + g[i];
      }
    }
  }
}

// Stable scatter of one tile by its segment's digit into the other buffer.
template <int TI, int NW, bool PERSIST>
__global__ __launch_bounds__(64 * NW) void k_level_scatter(const Seg *__restrict__ segs,
                                                         const uint32_t *__restrict__ tile_prefix,
                                                         const uint32_t *__restrict__ group_prefix, uint32_t nsegs,
                                                         const uint32_t *__restrict__ dev_nsegs,
                                                         const uint8_t *__restrict__ seg_split,
                                                         const uint32_t *__restrict__ tile_hist,
                                                         const uint32_t *__restrict__ gsum, uint64_t *keys0,
                                                         uint64_t *keys1, uint32_t *hdl0, uint32_t *hdl1) {
  constexpr uint32_t TL = 64 * NW * TI;
  __shared__ ScatterSmem<TI, NW> S;
  if (dev_nsegs) nsegs = *dev_nsegs;
  if (nsegs == 0) return;
  // virtual block v maps to a tile as a grid of ntiles would (neighbouring
  // tiles on one XCD); a persistent grid is a multiple of the XCD count, so
  // every workgroup stays on the XCD of its tiles
  const uint32_t ntiles = PERSIST ? tile_prefix[nsegs] : gridDim.x;
  for (uint32_t v = blockIdx.x; v < ntiles; v += gridDim.x) {
  const uint32_t tile = xcd_tile(v, ntiles);
  const uint32_t s = find_upper(tile_prefix, nsegs, tile);
  if (!seg_split[s]) {
    if (!PERSIST) break;
    continue;
  }
  if (PERSIST) __syncthreads();  // the previous tile's LDS reads are done
  const Seg sg = segs[s];
  const uint32_t tl = tile - tile_prefix[s];
  const uint64_t t0 = sg.start + (uint64_t)tl * TL;
  const uint32_t m = (uint32_t)min((uint64_t)TL, sg.start + sg.len - t0);
  const uint64_t *Ki = sg.buf ? keys1 : keys0;
  const uint32_t *Hi = sg.buf ? hdl1 : hdl0;
  uint64_t *Ko = sg.buf ? keys0 : keys1;
  uint32_t *Ho = sg.buf ? hdl0 : hdl1;
  const int d = sg.d;
  uint64_t kr[TI];
  uint32_t hr[TI], dig[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const uint32_t li = item_index<TI>(i);
    if (li < m) {
      kr[i] = Ki[t0 + li];
      hr[i] = Hi[t0 + li];
      dig[i] = digit_of(kr[i], d);
    } else {
      kr[i] = 0;
      hr[i] = 0;
      dig[i] = NODIGIT;
    }
  }
  const uint32_t g = group_prefix[s] + tl / GROUP_TILES;
  if (threadIdx.x < 256)
    S.goff[threadIdx.x] =
        (uint64_t)gsum[(uint64_t)g * 256 + threadIdx.x] + tile_hist[(uint64_t)tile * 256 + threadIdx.x];
  tile_scatter(S, kr, hr, dig, m, d, Ko, Ho);
  if (!PERSIST) break;
  }
}

// Groups of identical suffixes too large for one workgroup: emit in place.
template <bool PERSIST>
__global__ __launch_bounds__(BLOCK) void k_emit_final(const Seg *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                                                      uint32_t nsegs, const uint32_t *__restrict__ dev_nsegs,
                                                      uint32_t tile_len, const uint64_t *__restrict__ keys0,
                                                      const uint64_t *__restrict__ keys1, const uint32_t *__restrict__ hdl0,
                                                      const uint32_t *__restrict__ hdl1, const TextRec *__restrict__ text,
                                                      const uint32_t *__restrict__ srank,
                                                      const CollMap *__restrict__ cmap, uint8_t *__restrict__ bwt,
                                                      uint64_t *__restrict__ start_row) {
  if (dev_nsegs) nsegs = *dev_nsegs;
  if (nsegs == 0) return;
  const uint32_t ntiles = PERSIST ? tile_prefix[nsegs] : blockIdx.x + 1;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t s = find_upper(tile_prefix, nsegs, tile);
    const Seg sg = segs[s];
    const uint64_t t0 = sg.start + (uint64_t)(tile - tile_prefix[s]) * tile_len;
    const uint64_t t1 = min(t0 + (uint64_t)tile_len, sg.start + sg.len);
    const uint64_t *K = sg.buf ? keys1 : keys0;
    const uint32_t *H = sg.buf ? hdl1 : hdl0;
    const CollMap cm = cmap[sg.coll];
    for (uint64_t j = t0 + threadIdx.x; j < t1; j += BLOCK) emit_row(j, cm, K[j], H[j], text, srank, bwt, start_row);
    if (!PERSIST) break;
  }
}

// ---------------------------------------------------------------------------
// a2/a3/a4 in one wave: finish a chunk of at most 64 LI suffixes in LDS.
// A chunk is small enough that every group in it is ranked by all-pairs
// comparison, so the kernel needs no multisplit and no cross-wave barrier;
// many independent one-wave workgroups per CU hide each other's latency.
// Each round works on the list of live positions only (the members of
// groups that are not finished), so the rounds that refine a few tied
// groups cost little.
// ---------------------------------------------------------------------------
template <int LI>
struct LocalSmem {
  static constexpr int CHUNK = LOCAL_WG * LI;
  uint64_t K[CHUNK];  // key of each position
  uint32_t H[CHUNK];  // handle of each position
  union {
    struct {
      uint16_t live[CHUNK];    // live positions, ascending
      uint16_t gr[CHUNK];      // group of each live-list entry
      uint16_t hp[CHUNK + 1];  // first live-list entry of each group
      uint16_t dst[CHUNK];     // new position of each live-list entry
    };
    struct {                   // while the chunk is split by digits
      uint32_t cnt[256];
      uint32_t dstart[256];
    };
  };
  uint8_t head[CHUNK];  // position starts a group
};

constexpr int FETCH_BATCH = 2;  // window loads in flight per lane

// Stable split of the m suffixes of a chunk by 8-bit digit sel, in place
// (every suffix is held in registers before any moves).
template <int LI>
__device__ __forceinline__ void wave_split(LocalSmem<LI> &S, uint32_t m, int sel, uint32_t lane, uint64_t lt) {
  for (uint32_t x = lane; x < 256; x += LOCAL_WG) S.cnt[x] = 0;
  __syncthreads();
  uint64_t kr[LI];
  uint32_t hr[LI], dig[LI], pos[LI];
#pragma unroll
  for (int i = 0; i < LI; ++i) {
    const uint32_t j = i * LOCAL_WG + lane;
    const bool valid = j < m;
    dig[i] = NODIGIT;
    if (valid) {
      kr[i] = S.K[j];
      hr[i] = S.H[j];
      dig[i] = digit_of(kr[i], sel);
    }
    if (i * LOCAL_WG >= (int)m) continue;
    // rank among the lanes of this slot with the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig[i] >> b) & 1u;
      const uint64_t v = __ballot(bit);
      peers &= bit ? v : ~v;
    }
    if (valid) {
      const uint32_t before = S.cnt[dig[i]];
      pos[i] = before + (uint32_t)__popcll(peers & lt);
      if ((peers & lt) == 0) S.cnt[dig[i]] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
  }
  // digit starts: lane l sums digits 4l .. 4l+3
  const uint32_t c0 = S.cnt[4 * lane], c1 = S.cnt[4 * lane + 1], c2 = S.cnt[4 * lane + 2], c3 = S.cnt[4 * lane + 3];
  const uint32_t tot = c0 + c1 + c2 + c3;
  const uint32_t ex = wave_incl_sum(tot) - tot;
  S.dstart[4 * lane] = ex;
  S.dstart[4 * lane + 1] = ex + c0;
  S.dstart[4 * lane + 2] = ex + c0 + c1;
  S.dstart[4 * lane + 3] = ex + c0 + c1 + c2;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < LI; ++i) {
    if (dig[i] != NODIGIT) {
      const uint32_t q = S.dstart[dig[i]] + pos[i];
      S.K[q] = kr[i];
      S.H[q] = hr[i];
    }
  }
  __syncthreads();
}

// Groups of the live list from the head flags of its positions: gr[x] and
// hp[g] (hp[number of groups] = n).  One ballot per 64 entries.
template <int LI>
__device__ __forceinline__ void live_groups(LocalSmem<LI> &S, uint32_t n, uint32_t lane, uint64_t le) {
  uint32_t run = 0;
#pragma unroll
  for (int i = 0; i < LI; ++i) {
    const uint32_t x = i * LOCAL_WG + lane;
    if (i * LOCAL_WG >= (int)n) break;
    const bool in = x < n;
    const bool h = in && S.head[S.live[x]];
    const uint64_t hb = __ballot(h);
    const uint32_t g = run + (uint32_t)__popcll(hb & le) - 1u;
    if (in) {
      S.gr[x] = (uint16_t)g;
      if (h) S.hp[g] = (uint16_t)x;
    }
    run += (uint32_t)__popcll(hb);
  }
  if (lane == 0) S.hp[run] = (uint16_t)n;
  __syncthreads();
}

// LI suffixes per lane; OCC waves per SIMD the kernel is compiled for;
// PERSIST: a fixed grid loops over a chunk count on the device
template <int LI, int OCC, bool PERSIST>
__global__ __launch_bounds__(LOCAL_WG, OCC) void k_local(
    const Seg *__restrict__ chunks, const uint64_t *__restrict__ keys0, const uint64_t *__restrict__ keys1,
    const uint32_t *__restrict__ hdl0, const uint32_t *__restrict__ hdl1, const TextRec *__restrict__ text,
    const uint32_t *__restrict__ srank, const CollMap *__restrict__ cmap, uint64_t nb, uint32_t rmax,
    uint8_t *__restrict__ bwt, uint64_t *__restrict__ start_row, uint32_t *status, unsigned long long *fetches,
    uint32_t n_chunks, const uint32_t *__restrict__ dev_nchunks, uint32_t first) {
  __shared__ LocalSmem<LI> S;
  const uint32_t lane = threadIdx.x;
  const uint64_t le = lanemask_lt() | (1ull << lane);
  // chunks first + blockIdx.x (+ k * gridDim.x when PERSIST) below the count
  if (dev_nchunks) n_chunks = *dev_nchunks;
  uint32_t nfetch = 0;
  for (uint32_t c = first + blockIdx.x; c < n_chunks; c += gridDim.x) {
  if (PERSIST) __syncthreads();  // the previous chunk's LDS reads are done
  const Seg ch = chunks[c];
  const uint32_t m = (uint32_t)ch.len;
  const uint64_t *Kg = ch.buf ? keys1 : keys0;
  const uint32_t *Hg = ch.buf ? hdl1 : hdl0;
  // entry x of a list is handled by lane x % 64 in slot x / 64: neighbouring
  // lanes hold neighbouring positions, which mostly share a group
#pragma unroll
  for (int i = 0; i < LI; ++i) {
    const uint32_t j = i * LOCAL_WG + lane;
    if (j < m) {
      S.K[j] = Kg[ch.start + j];
      S.H[j] = Hg[ch.start + j];
    }
  }
  __syncthreads();
  // The chunk is a run of buckets that differ in digit d and agree before
  // it (or, unsplit, in read order, with d = 0).  Two stable splits, by digit
  // d + 1 and then by digit d, leave it ordered by both digits; the groups of
  // equal (d, d + 1) digits are then sorted on their current key, and after
  // that groups are runs of equal keys, refined window by window.
  const int d0 = ch.d;
  const bool two = d0 < 7;
  if (two) {
    wave_split(S, m, d0 + 1, lane, le & ~(1ull << lane));
    wave_split(S, m, d0, lane, le & ~(1ull << lane));
  }
#pragma unroll
  for (int i = 0; i < LI; ++i) {
    const uint32_t j = i * LOCAL_WG + lane;
    if (j < m) {
      bool h = j == 0;
      if (!h && two) h = digit_of(S.K[j], d0) != digit_of(S.K[j - 1], d0) ||
                         digit_of(S.K[j], d0 + 1) != digit_of(S.K[j - 1], d0 + 1);
      else if (!h) h = !ch.unsplit && digit_of(S.K[j], d0) != digit_of(S.K[j - 1], d0);
      S.head[j] = h;
      S.live[j] = (uint16_t)j;
    }
  }
  __syncthreads();
  uint32_t n = m;  // live-list length
  uint32_t r = ch.r;
  bool fetch_round = false;
  for (;;) {
    // drop the finished groups: single suffixes, and (after the first sort)
    // runs of equal keys that end inside the window, i.e. identical suffixes.
    // A group is a run of live entries from a head to the next head, so an
    // entry is alone in its group when it and the next live entry are both
    // heads; the other test is the same for every member of a group of
    // equal keys, so whole groups stay or go.
    uint32_t kept = 0;
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      if (i * LOCAL_WG >= (int)n) break;
      const uint32_t x = i * LOCAL_WG + lane;
      bool keep = false;
      uint16_t pos = 0;
      if (x < n) {
        pos = S.live[x];
        // entry x + 1 is read before any slot writes an index above x
        const bool alone = S.head[pos] && (x + 1 >= n || S.head[S.live[x + 1]]);
        keep = !alone && (!fetch_round || clamp_of(S.K[pos]) == (uint32_t)W);
      }
      const uint64_t kb = __ballot(keep);
      // compaction moves entries down only, so slot i never overwrites an
      // entry a later slot still has to read
      if (keep) S.live[kept + (uint32_t)__popcll(kb & (le >> 1))] = pos;
      kept += (uint32_t)__popcll(kb);
    }
    n = kept;
    if (n == 0) break;
    __syncthreads();
    live_groups(S, n, lane, le);
    if (fetch_round) {
      if (r + 1 > rmax) {
        if (lane == 0) atomicOr(status, ST_WINDOW_BOUND);
        break;
      }
      ++r;
      // fetch the next window of every live suffix, FETCH_BATCH loads in
      // flight per lane
      for (uint32_t x0 = 0; x0 < n; x0 += FETCH_BATCH * LOCAL_WG) {
        TextRec tr[FETCH_BATCH];
        uint32_t tp[FETCH_BATCH];
#pragma unroll
        for (int i = 0; i < FETCH_BATCH; ++i) {
          const uint32_t x = x0 + i * LOCAL_WG + lane;
          if (x < n) {
            tp[i] = S.live[x];
            tr[i] = window_load(text, nb, S.H[tp[i]], r);
          }
        }
#pragma unroll
        for (int i = 0; i < FETCH_BATCH; ++i) {
          const uint32_t x = x0 + i * LOCAL_WG + lane;
          if (x < n) {
            const uint32_t j = tp[i];
            S.K[j] = window_combine(tr[i], nb, S.H[j], r, (uint32_t)S.K[j] & 7u);
            ++nfetch;
          }
        }
      }
      __syncthreads();
    }
    // stable rank inside each live group by all-pairs comparison:
    // rank = #{t < j : key_t <= key_j} + #{t > j : key_t < key_j}; every
    // rank is taken before any entry moves.  The ordering bits oj are a
    // multiple of 8, so (key_t & ~7) <= oj is key_t < oj + 8 and
    // (key_t & ~7) < oj is key_t < oj: one 64-bit compare per key, on the
    // raw keys (t = j adds nothing to the second count).
    for (uint32_t x = lane; x < n; x += LOCAL_WG) {
      const uint32_t j = S.live[x];
      const uint32_t g = S.gr[x];
      const uint32_t x0 = S.hp[g];
      const uint32_t a = S.live[x0];
      const uint32_t e = a + ((uint32_t)S.hp[g + 1] - x0);  // a group is a run of positions
      const uint64_t oj = order_bits(S.K[j]);
      const uint64_t below = oj + 8;  // cannot wrap: key bits 9..8 are zero
      // four independent LDS reads per step keep the loops off the
      // load-latency chain
      uint32_t c = 0;
      uint32_t t = a;
      for (; t + 4 <= j; t += 4)
        c += (uint32_t)(S.K[t] < below) + (uint32_t)(S.K[t + 1] < below) + (uint32_t)(S.K[t + 2] < below) +
             (uint32_t)(S.K[t + 3] < below);
      for (; t < j; ++t) c += (uint32_t)(S.K[t] < below);
      for (; t + 4 <= e; t += 4)
        c += (uint32_t)(S.K[t] < oj) + (uint32_t)(S.K[t + 1] < oj) + (uint32_t)(S.K[t + 2] < oj) +
             (uint32_t)(S.K[t + 3] < oj);
      for (; t < e; ++t) c += (uint32_t)(S.K[t] < oj);
      S.dst[x] = (uint16_t)(a + c);
    }
    __syncthreads();
    {
      uint64_t sk[LI];
      uint32_t sh[LI], sd[LI];
#pragma unroll
      for (int i = 0; i < LI; ++i) {
        const uint32_t x = i * LOCAL_WG + lane;
        if (x < n) {
          const uint32_t j = S.live[x];
          sk[i] = S.K[j];
          sh[i] = S.H[j];
          sd[i] = S.dst[x];
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < LI; ++i) {
        const uint32_t x = i * LOCAL_WG + lane;
        if (x < n) {
          S.K[sd[i]] = sk[i];
          S.H[sd[i]] = sh[i];
        }
      }
    }
    __syncthreads();
    // new group heads inside live groups: changes of the full key
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      const uint32_t x = i * LOCAL_WG + lane;
      if (i * LOCAL_WG >= (int)n) break;
      if (x >= n) continue;
      const uint32_t j = S.live[x];
      if (!S.head[j] && order_bits(S.K[j]) != order_bits(S.K[j - 1])) S.head[j] = 1;
    }
    __syncthreads();
    fetch_round = true;
  }
  // a4: emit
  const CollMap cm = cmap[ch.coll];
#pragma unroll
  for (int i = 0; i < LI; ++i) {
    const uint32_t j = i * LOCAL_WG + lane;
    if (j < m) emit_row(ch.start + j, cm, S.K[j], S.H[j], text, srank, bwt, start_row);
  }
  if (!PERSIST) break;
  }
  nfetch = wave_incl_sum(nfetch);
  if (lane == 63 && nfetch) atomicAdd(stat_slot(fetches), (unsigned long long)nfetch);
}


// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
thread_local cxbwt_stats g_stats;
thread_local int g_timing = 0;

// The instantiation a build uses (see the tuning constants).
struct Tuning {
  uint32_t tile_items;   // 6, 8 or 16 suffixes per 256 threads' thread in a level tile (16: 8 waves x 8)
  uint32_t chunk_items;  // 3, 6 or 8 suffixes per lane in a chunk
  uint32_t tile_len() const { return BLOCK * tile_items; }
  uint32_t chunk() const { return LOCAL_WG * chunk_items; }
};
thread_local Tuning g_tuning{8, 6};

// tile_items 16 is the wide tile: 8 waves x 8 items (4096 suffixes); the
// histogram kernels take it as two sub-tiles of BLOCK * MAX_TILE_ITEMS
static_assert(BLOCK * MAX_TILE_ITEMS * 2 == 4096, "a wide tile is two histogram sub-tiles");
bool tuning_ok(uint32_t tile_items, uint32_t chunk_items) {
  return (tile_items == 6 || tile_items == 8 || tile_items == 16) &&
         (chunk_items == 3 || chunk_items == 6 || chunk_items == 8);
}

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t align_up(uint64_t x) { return (x + 255) & ~255ull; }


struct Layout {
  uint64_t keys0, keys1, hdl0, hdl1, text, srank, rank_blocks, start_row, tile_hist, gsum, segs, tile_prefix,
      group_prefix, seg_or, seg_and, seg_split, big_next, chunks, finals, coll_reads, coll_bases, cmap, counters,
      stats, total;
  uint64_t cap_big, cap_chunks, cap_finals, seg_slots, max_tiles, max_groups, n_rec, n_rank_words, n_rank_blocks;
};

bool sizes_ok(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len) {
  return n_reads >= 1 && n_reads < (1ull << 32) && n_bases <= CXBWT_MAX_BASES && max_read_len <= CXBWT_MAX_READ_LEN;
}

Layout make_layout(uint64_t n_reads, uint64_t nb, uint32_t n_coll) {
  Layout L{};
  // segments of one level are disjoint and each holds more than a chunk
  // (at least MIN_CHUNK) suffixes; level 1 starts with one segment per
  // collection
  L.cap_big = nb / (MIN_CHUNK + 1) + 2;
  L.cap_finals = L.cap_big;
  // chunks of one level: two neighbouring chunks of a run hold more than
  // a chunk's suffixes together, and a run ends at an oversized bucket or at the
  // end of its parent (both at most cap_big per level); level 1 adds one
  // chunk per collection that fits a chunk
  L.cap_chunks = 2 * ceil_div(nb, MIN_CHUNK) + 2 * L.cap_big + n_coll + 2;
  // segments split in one batch of a level: the per-segment and per-tile
  // scratch is sized for segments of more than SEG_BATCH_MIN suffixes; a
  // level with more segments runs in several batches.  Level 1 (one segment
  // per collection) always fits one batch.
  L.seg_slots = std::max<uint64_t>(nb / (SEG_BATCH_MIN + 1) + 2, (uint64_t)n_coll + 1);
  L.max_tiles = ceil_div(nb, MIN_TILE) + L.seg_slots + 1;
  L.max_groups = ceil_div(nb, (uint64_t)MIN_TILE * GROUP_TILES) + L.seg_slots + 1;
  L.n_rec = nb / 16 + 2;
  L.n_rank_words = ceil_div(L.n_rec, 2);  // bitmap words covering the records
  L.n_rank_blocks = ceil_div(L.n_rank_words, RANK_BLOCK_WORDS);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const uint64_t seg_slots = L.seg_slots;
  L.keys0 = take(8 * nb);
  L.keys1 = take(8 * nb);
  L.hdl0 = take(4 * nb);
  L.hdl1 = take(4 * nb);
  L.text = take(sizeof(TextRec) * L.n_rec);
  L.srank = take(4 * L.n_rec);
  L.rank_blocks = take(4 * L.n_rank_blocks);
  L.start_row = take(8 * n_reads);
  L.tile_hist = take(4 * 256 * L.max_tiles);
  L.gsum = take(4 * 256 * L.max_groups);
  L.segs = take(sizeof(Seg) * seg_slots);
  // tile prefixes serve a batch of segments and, after it, the final groups
  // of the batch (each more than a chunk's suffixes: at most cap_finals)
  L.tile_prefix = take(4 * (std::max(seg_slots, L.cap_finals) + 1));
  L.group_prefix = take(4 * (seg_slots + 1));
  L.seg_or = take(8 * seg_slots);
  L.seg_and = take(8 * seg_slots);
  L.seg_split = take(seg_slots);
  L.big_next = take(sizeof(Seg) * L.cap_big);
  L.chunks = take(sizeof(Seg) * L.cap_chunks);
  L.finals = take(sizeof(Seg) * L.cap_finals);
  L.coll_reads = take(8 * ((uint64_t)n_coll + 1));
  L.coll_bases = take(8 * ((uint64_t)n_coll + 1));
  L.cmap = take(sizeof(CollMap) * (uint64_t)n_coll);
  L.counters = take(4 * C_COUNT);
  L.stats = take(8 * STAT_WORDS);
  L.total = off;
  return L;
}

#define CX_CHECK(x)                              \
  do {                                           \
    if ((x) != hipSuccess) return CXBWT_EDEVICE; \
  } while (0)
#define CX_LAUNCHED()                                          \
  do {                                                         \
    if (hipGetLastError() != hipSuccess) return CXBWT_EDEVICE; \
  } while (0)

unsigned grid_for(uint64_t n, unsigned block) {
  uint64_t g = ceil_div(n, block);
  if (g == 0) g = 1;
  if (g > 0x7FFFFFFFull) g = 0x7FFFFFFFull;
  return (unsigned)g;
}

int fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st) {
  if (!n) return CXBWT_OK;
  unsigned g = grid_for(n, 256);
  if (g > 65536) g = 65536;
  k_fill_u64<<<g, 256, 0, st>>>(p, n, v);
  CX_LAUNCHED();
  return CXBWT_OK;
}
int fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) {
  if (!n) return CXBWT_OK;
  unsigned g = grid_for(n, 256);
  if (g > 65536) g = 65536;
  k_fill_u32<<<g, 256, 0, st>>>(p, n, v);
  CX_LAUNCHED();
  return CXBWT_OK;
}

// Kernel classes timed by PhaseTimer (indices of cxbwt_stats.ms).
enum Phase { PH_PREP = 0, PH_GEN, PH_HIST, PH_SCAN, PH_SCATTER, PH_LOCAL, PH_FINAL };

// Brackets kernel launches with HIP events on the build's stream when timing
// is on; durations are summed at the host synchronisation points.
struct PhaseTimer {
  hipStream_t st;
  bool on;
  struct Pending {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  hipEvent_t open_ev = nullptr;
  static std::vector<hipEvent_t> &pool() {
    thread_local std::vector<hipEvent_t> p;
    return p;
  }
  hipEvent_t get() {
    auto &p = pool();
    if (!p.empty()) {
      hipEvent_t e = p.back();
      p.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin() {
    if (!on) return;
    open_ev = get();
    if (open_ev) (void)hipEventRecord(open_ev, st);
  }
  void end(int phase) {
    if (!on || !open_ev) return;
    hipEvent_t b = get();
    if (!b) return;
    (void)hipEventRecord(b, st);
    pending.push_back({phase, open_ev, b});
    open_ev = nullptr;
  }
  // call only after the stream has been synchronised
  void collect() {
    for (auto &q : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) g_stats.ms[q.phase] += ms;
      g_stats.launches[q.phase]++;
      pool().push_back(q.a);
      pool().push_back(q.b);
    }
    pending.clear();
  }
  ~PhaseTimer() {
    for (auto &q : pending) {
      pool().push_back(q.a);
      pool().push_back(q.b);
    }
    if (open_ev) pool().push_back(open_ev);
  }
};


struct Buffers {
  uint64_t *keys0, *keys1, *start_row, *coll_reads, *coll_bases;
  TextRec *text;
  uint32_t *hdl0, *hdl1, *srank, *rank_blocks, *tile_hist, *gsum, *tile_prefix, *group_prefix, *counters;
  Seg *segs, *big_next, *chunks, *finals;
  CollMap *cmap;
  unsigned long long *seg_or, *seg_and, *stats;
  uint8_t *seg_split;
};

// End of the batch of segments starting at b0 that fits the per-segment and
// per-tile scratch (at least one segment: a single segment always fits).
size_t batch_end(const std::vector<Seg> &segs, size_t b0, const Layout &Lo, uint32_t tile_len) {
  uint64_t tiles = 0, groups = 0;
  size_t b1 = b0;
  while (b1 < segs.size() && b1 - b0 < Lo.seg_slots) {
    const uint64_t nt = ceil_div(segs[b1].len, tile_len);
    const uint64_t ng = ceil_div(nt, GROUP_TILES);
    if (b1 > b0 && (tiles + nt > Lo.max_tiles || groups + ng > Lo.max_groups)) break;
    tiles += nt;
    groups += ng;
    ++b1;
  }
  return b1;
}

// Upload a segment list with its tile and group prefixes; returns the tile
// and group totals.
int upload_segments(const Buffers &B, const Layout &Lo, const std::vector<Seg> &segs, uint32_t tile_len,
                    std::vector<uint32_t> &tprefix, std::vector<uint32_t> &gprefix, uint32_t &ntiles,
                    uint32_t &ngroups, hipStream_t st) {
  const uint32_t ns = (uint32_t)segs.size();
  if (ns > Lo.seg_slots) return CXBWT_EDEVICE;
  tprefix.assign(ns + 1, 0);
  gprefix.assign(ns + 1, 0);
  for (uint32_t i = 0; i < ns; ++i) {
    const uint32_t nt = (uint32_t)ceil_div(segs[i].len, tile_len);
    tprefix[i + 1] = tprefix[i] + nt;
    gprefix[i + 1] = gprefix[i] + (uint32_t)ceil_div(nt, GROUP_TILES);
  }
  ntiles = tprefix[ns];
  ngroups = gprefix[ns];
  if (ntiles > Lo.max_tiles || ngroups > Lo.max_groups) return CXBWT_EDEVICE;
  CX_CHECK(hipMemcpyAsync(B.segs, segs.data(), sizeof(Seg) * ns, hipMemcpyHostToDevice, st));
  CX_CHECK(hipMemcpyAsync(B.tile_prefix, tprefix.data(), 4 * (ns + 1), hipMemcpyHostToDevice, st));
  CX_CHECK(hipMemcpyAsync(B.group_prefix, gprefix.data(), 4 * (ns + 1), hipMemcpyHostToDevice, st));
  return CXBWT_OK;
}

// Workgroups of the launches whose size is fixed before their work count is
// known (the work count is read on the device; see the kernels): a few per
// CU, multiples of the XCD count.
constexpr unsigned PG_HIST = 256 * 8;
constexpr unsigned PG_GROUP = 256 * 4;
constexpr unsigned PG_SCAN = 256 * 4;
constexpr unsigned PG_SCATTER = 256 * 5;
constexpr unsigned PG_SCATTER_WIDE = 256 * 2;
constexpr unsigned PG_EMIT = 256 * 4;
constexpr unsigned PG_FILL = 256 * 2;

// Second scan stage launch: a workgroup per segment when the segments span
// many groups each (the first levels), else a wave per segment.  With
// dev_ns the count is on the device and the launch is the fixed one of a
// wave per segment.
void launch_level_scan(const Buffers &B, uint32_t ns, uint32_t ngroups, const Lists &Ls, int force_split,
                       hipStream_t st, const uint32_t *dev_ns = nullptr, unsigned dev_grid = PG_SCAN) {
  if (dev_ns)
    k_level_scan<false, true><<<dev_grid, BLOCK, 0, st>>>(B.segs, B.group_prefix, 0, B.gsum, B.seg_or, B.seg_and,
                                                   B.seg_split, Ls, force_split, dev_ns);
  else if (ngroups > 8u * ns)
    k_level_scan<true, false><<<ns, BLOCK, 0, st>>>(B.segs, B.group_prefix, ns, B.gsum, B.seg_or, B.seg_and, B.seg_split,
                                             Ls, force_split, nullptr);
  else
    k_level_scan<false, false><<<(unsigned)ceil_div(ns, WAVES), BLOCK, 0, st>>>(B.segs, B.group_prefix, ns, B.gsum,
                                                                          B.seg_or, B.seg_and, B.seg_split, Ls,
                                                                          force_split, nullptr);
}

// Tile prefixes (and group prefixes, and a copy of the list, when given) of
// the first n entries of a segment list, computed on the device.  Uses the
// scan-group totals area as scratch.  With dev_n the count is on the device
// and n is only its bound.
int prefix_list(const Buffers &B, const Seg *list, uint32_t n, uint32_t tile_len, Seg *copy, uint32_t *tprefix,
                uint32_t *gprefix, hipStream_t st, const uint32_t *dev_n = nullptr) {
  if (!n) return CXBWT_OK;
  const unsigned nwg = (unsigned)ceil_div(n, SEGP_WG);
  k_seg_count<<<nwg, BLOCK, 0, st>>>(list, n, dev_n, tile_len, B.gsum);
  CX_LAUNCHED();
  k_seg_scan<<<nwg, BLOCK, 0, st>>>(list, n, dev_n, tile_len, B.gsum, copy, tprefix, gprefix);
  CX_LAUNCHED();
  return CXBWT_OK;
}

// What one scan of a level handed on, from the counters block after the
// fold.
struct LevelOut {
  uint32_t status, n_chunks, n_finals, n_big;  // n_big: all batches of the level so far
  uint64_t next_len, next_regather, next_maxr, next_tiles, next_groups, final_len, final_tiles;
};

// Fold the level statistics, read the counters back (the one wait of a
// level batch).
int read_level(const Buffers &B, LevelOut &o, PhaseTimer &T, hipStream_t st) {
  uint32_t hc[C_COUNT];
  k_level_fold<<<1, 64, 0, st>>>(B.stats, (unsigned long long *)(B.counters + C_FOLD), nullptr);
  CX_LAUNCHED();
  CX_CHECK(hipMemcpyAsync(hc, B.counters, sizeof(hc), hipMemcpyDeviceToHost, st));
  CX_CHECK(hipStreamSynchronize(st));
  T.collect();
  uint64_t f[K_LEVEL_KINDS];
  memcpy(f, hc + C_FOLD, sizeof(f));
  o.status = hc[C_STATUS];
  o.n_chunks = hc[C_NCHUNK];
  o.n_finals = hc[C_NFINAL];
  o.n_big = hc[C_NBIG];
  o.next_len = f[K_NEXT_LEN - K_LEVEL_FIRST];
  o.next_regather = f[K_NEXT_REGATHER - K_LEVEL_FIRST];
  o.next_maxr = f[K_NEXT_MAXR - K_LEVEL_FIRST];
  o.next_tiles = f[K_NEXT_TILES - K_LEVEL_FIRST];
  o.next_groups = f[K_NEXT_GROUPS - K_LEVEL_FIRST];
  o.final_len = f[K_FINAL_LEN - K_LEVEL_FIRST];
  o.final_tiles = f[K_FINAL_TILES - K_LEVEL_FIRST];
  return o.status ? CXBWT_EDEVICE : CXBWT_OK;
}

// Work counts of one level as an eager build saw them (level 1 at index 0).
// A captured build sizes its launches from them, so that each workgroup
// usually takes one item as in an eager launch (the looping kernels stay
// correct for larger counts).
struct LevelShape {
  uint32_t nsegs = 0, ntiles = 0, ngroups = 0, nchunks = 0, nfinals = 0, ftiles = 0;
};
thread_local std::vector<LevelShape> *g_shapes = nullptr;  // recorder of an eager build, when set

void record_shape(uint32_t level, const LevelShape &x) {
  if (!g_shapes) return;
  if (g_shapes->size() <= level) g_shapes->resize(level + 1);
  LevelShape &y = (*g_shapes)[level];
  y.nsegs = std::max(y.nsegs, x.nsegs);
  y.ntiles = std::max(y.ntiles, x.ntiles);
  y.ngroups = std::max(y.ngroups, x.ngroups);
  y.nchunks = std::max(y.nchunks, x.nchunks);
  y.nfinals = std::max(y.nfinals, x.nfinals);
  y.ftiles = std::max(y.ftiles, x.ftiles);
}

// Launch size for an item count seen before: a quarter more, a multiple of
// the XCD count, or the fixed size when nothing was seen.
unsigned grid_from(uint32_t seen, unsigned fixed) {
  if (!seen) return fixed;
  const uint64_t g = ((uint64_t)seen + seen / 4 + 64 + 7) & ~7ull;
  return (unsigned)std::min<uint64_t>(g, 0x7FFFFFF8ull);
}

// The chunk kernel for the selected chunk size: one workgroup per chunk, or
// with dev_nchunks a launch of `grid` workgroups (0: a few waves per SIMD)
// looping over a count on the device.
int launch_local(const Buffers &B, const Tuning &tu, uint64_t nb, uint32_t rmax, uint8_t *bwt, uint32_t n_chunks,
                 const uint32_t *dev_nchunks, hipStream_t st, unsigned grid = 0) {
  // the looping form holds a few more registers: one wave per SIMD fewer
  // for the smallest chunk keeps it from spilling
  // with a device count and a grid: the one-chunk form over the first
  // `grid` chunks, then the looping form over any beyond them
#define CX_LOCAL(LI, OCC, OCCP)                                                                                  \
  do {                                                                                                           \
    if (dev_nchunks && grid) {                                                                                   \
      k_local<LI, OCC, false><<<grid, LOCAL_WG, 0, st>>>(B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.text,      \
                                                        B.srank, B.cmap, nb, rmax, bwt, B.start_row,             \
                                                        B.counters + C_STATUS, B.stats, 0, dev_nchunks, 0);      \
      k_local<LI, OCCP, true><<<256u, LOCAL_WG, 0, st>>>(B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.text,      \
                                                        B.srank, B.cmap, nb, rmax, bwt, B.start_row,             \
                                                        B.counters + C_STATUS, B.stats, 0, dev_nchunks, grid);   \
    } else if (dev_nchunks) {                                                                                    \
      k_local<LI, OCCP, true><<<256u * 4u * OCCP, LOCAL_WG, 0, st>>>(                                            \
          B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.text, B.srank, B.cmap, nb, rmax, bwt, B.start_row,      \
          B.counters + C_STATUS, B.stats, 0, dev_nchunks, 0);                                                    \
    } else {                                                                                                     \
      k_local<LI, OCC, false><<<n_chunks, LOCAL_WG, 0, st>>>(B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.text, \
                                                            B.srank, B.cmap, nb, rmax, bwt, B.start_row,         \
                                                            B.counters + C_STATUS, B.stats, n_chunks, nullptr,   \
                                                            0);                                                  \
    }                                                                                                            \
  } while (0)
  if (tu.chunk_items == 8) CX_LOCAL(8, 3, 3);
  else if (tu.chunk_items == 6) CX_LOCAL(6, 4, 4);
  else CX_LOCAL(3, 6, 5);
#undef CX_LOCAL
  CX_LAUNCHED();
  return CXBWT_OK;
}

// Finish the chunks and final groups a level produced.
int finish_level(const Buffers &B, const Layout &Lo, const Tuning &tu, uint64_t nb, uint32_t rmax, uint8_t *bwt,
                 uint32_t n_chunks, uint32_t n_finals, uint64_t final_tiles, uint64_t final_len, PhaseTimer &T,
                 hipStream_t st) {
  if (n_chunks > Lo.cap_chunks || n_finals > Lo.cap_finals) return CXBWT_EDEVICE;
  int rc;
  if (n_chunks) {
    T.begin();
    if ((rc = launch_local(B, tu, nb, rmax, bwt, n_chunks, nullptr, st))) return rc;
    T.end(PH_LOCAL);
    g_stats.chunks += n_chunks;
  }
  if (n_finals) {
    if (final_tiles == 0 || final_tiles > 0xFFFFFFFFull) return CXBWT_EDEVICE;
    if ((rc = prefix_list(B, B.finals, n_finals, tu.tile_len(), nullptr, B.tile_prefix, nullptr, st))) return rc;
    T.begin();
    k_emit_final<false><<<(unsigned)final_tiles, BLOCK, 0, st>>>(B.finals, B.tile_prefix, n_finals, nullptr, tu.tile_len(),
                                                          B.keys0, B.keys1, B.hdl0, B.hdl1, B.text, B.srank, B.cmap,
                                                          bwt, B.start_row);
    CX_LAUNCHED();
    T.end(PH_FINAL);
    g_stats.final_big += n_finals;
    g_stats.chunk_suffixes -= final_len;
  }
  return CXBWT_OK;
}

// Histogram, two scan stages and scatter of a level 2.. over nsg segments
// (ntiles tiles, ngroups groups), or with dev_nsg over a segment count on
// the device in launches of fixed size.
int launch_level_kernels(const Buffers &B, const Tuning &tu, const Lists &Ls, uint64_t nb, uint32_t nsg,
                         uint32_t ntiles, uint32_t ngroups, const uint32_t *dev_nsg, PhaseTimer &T, hipStream_t st,
                         const LevelShape *seen = nullptr) {
  const bool dev = dev_nsg != nullptr;
  // device mode: launch sizes from the counts seen, else fixed
  const LevelShape none;
  const LevelShape &sh = seen ? *seen : none;
  const unsigned g_hist = grid_from(sh.ntiles, PG_HIST), g_group = grid_from(sh.ngroups, PG_GROUP),
                 g_scan = grid_from((sh.nsegs + WAVES - 1) / WAVES, PG_SCAN),
                 g_scatter = grid_from(sh.ntiles, tu.tile_items == 16 ? PG_SCATTER_WIDE : PG_SCATTER);
  T.begin();
#define CX_HIST(P, SUBT)                                                                                         \
  k_level_hist<P, SUBT><<<P ? g_hist : ntiles, BLOCK, 0, st>>>(B.segs, B.tile_prefix, nsg, dev_nsg, tu.tile_len(),  \
                                                                B.keys0, B.keys1, B.hdl0, B.hdl1, B.text, nb,        \
                                                                B.tile_hist, B.seg_or, B.seg_and)
  if (tu.tile_items == 16) {
    if (dev) CX_HIST(true, 2);
    else CX_HIST(false, 2);
  } else {
    if (dev) CX_HIST(true, 1);
    else CX_HIST(false, 1);
  }
#undef CX_HIST
  CX_LAUNCHED();
  T.end(PH_HIST);
  T.begin();
  if (dev)
    k_group_scan<true><<<g_group, BLOCK, 0, st>>>(B.tile_prefix, B.group_prefix, nsg, dev_nsg, B.tile_hist, B.gsum);
  else
    k_group_scan<false><<<ngroups, BLOCK, 0, st>>>(B.tile_prefix, B.group_prefix, nsg, nullptr, B.tile_hist, B.gsum);
  CX_LAUNCHED();
  launch_level_scan(B, nsg, ngroups, Ls, 0, st, dev_nsg, g_scan);
  CX_LAUNCHED();
  T.end(PH_SCAN);
  T.begin();
#define CX_SCATTER(TI, NW, P)                                                                                   \
  k_level_scatter<TI, NW, P><<<P ? g_scatter : ntiles, 64 * NW, 0, st>>>(                                       \
      B.segs, B.tile_prefix, B.group_prefix, nsg, dev_nsg, B.seg_split, B.tile_hist, B.gsum, B.keys0, B.keys1,    \
      B.hdl0, B.hdl1)
  if (tu.tile_items == 16) {
    if (dev) CX_SCATTER(8, 8, true);
    else CX_SCATTER(8, 8, false);
  } else if (tu.tile_items == 8) {
    if (dev) CX_SCATTER(8, 4, true);
    else CX_SCATTER(8, 4, false);
  } else {
    if (dev) CX_SCATTER(6, 4, true);
    else CX_SCATTER(6, 4, false);
  }
#undef CX_SCATTER
  CX_LAUNCHED();
  T.end(PH_SCATTER);
  return CXBWT_OK;
}

// One batch of a level 2..: nsg segments in B.segs with their tile and group
// prefixes in place.  Counts, splits, scatters, then finishes the chunks and
// final groups the batch produced.
int run_level_batch(const Buffers &B, const Layout &Lo, const Tuning &tu, const Lists &Ls, uint64_t nb,
                    uint32_t rmax, uint8_t *bwt, uint32_t nsg, uint32_t ntiles, uint32_t ngroups, LevelOut &o,
                    PhaseTimer &T, hipStream_t st) {
  int rc;
  if ((rc = fill_u64((uint64_t *)B.seg_or, nsg, 0, st))) return rc;
  if ((rc = fill_u64((uint64_t *)B.seg_and, nsg, ~0ull, st))) return rc;
  if ((rc = fill_u32(B.counters + C_NFINAL, 2, 0, st))) return rc;  // final and chunk counts
  T.begin();
  if ((rc = launch_level_kernels(B, tu, Ls, nb, nsg, ntiles, ngroups, nullptr, T, st))) return rc;
  g_stats.level_batches++;
  if ((rc = read_level(B, o, T, st))) return rc;
  return finish_level(B, Lo, tu, nb, rmax, bwt, o.n_chunks, o.n_finals, o.final_tiles, o.final_len, T, st);
}

// Everything one build needs: its sizes, the caller's buffers, the workspace
// layout and the level-1 plan made from the collection bases.
struct Build {
  const uint64_t *packed, *offsets;
  uint64_t n, nb;
  uint32_t maxlen, ncoll;
  uint8_t *bwt;
  uint64_t *term_pos;
  Layout Lo;
  Buffers B;
  Tuning tu;
  uint32_t rmax, tile_len;
  Lists Ls;
  std::vector<uint64_t> coll_reads, cbase;
  std::vector<CollMap> cm;
  std::vector<Seg> big, small;  // level-1 segments; collections that fit one chunk
};

Buffers buffers_of(unsigned char *ws, const Layout &Lo) {
  Buffers B;
  B.keys0 = (uint64_t *)(ws + Lo.keys0);
  B.keys1 = (uint64_t *)(ws + Lo.keys1);
  B.hdl0 = (uint32_t *)(ws + Lo.hdl0);
  B.hdl1 = (uint32_t *)(ws + Lo.hdl1);
  B.text = (TextRec *)(ws + Lo.text);
  B.srank = (uint32_t *)(ws + Lo.srank);
  B.rank_blocks = (uint32_t *)(ws + Lo.rank_blocks);
  B.start_row = (uint64_t *)(ws + Lo.start_row);
  B.tile_hist = (uint32_t *)(ws + Lo.tile_hist);
  B.gsum = (uint32_t *)(ws + Lo.gsum);
  B.segs = (Seg *)(ws + Lo.segs);
  B.tile_prefix = (uint32_t *)(ws + Lo.tile_prefix);
  B.group_prefix = (uint32_t *)(ws + Lo.group_prefix);
  B.seg_or = (unsigned long long *)(ws + Lo.seg_or);
  B.seg_and = (unsigned long long *)(ws + Lo.seg_and);
  B.seg_split = (uint8_t *)(ws + Lo.seg_split);
  B.big_next = (Seg *)(ws + Lo.big_next);
  B.chunks = (Seg *)(ws + Lo.chunks);
  B.finals = (Seg *)(ws + Lo.finals);
  B.coll_reads = (uint64_t *)(ws + Lo.coll_reads);
  B.coll_bases = (uint64_t *)(ws + Lo.coll_bases);
  B.cmap = (CollMap *)(ws + Lo.cmap);
  B.counters = (uint32_t *)(ws + Lo.counters);
  B.stats = (unsigned long long *)(ws + Lo.stats);
  return B;
}

void build_init(Build &b, const uint64_t *packed, const uint64_t *offsets, uint64_t n, uint64_t nb, uint32_t maxlen,
                const uint64_t *coll_reads, uint32_t ncoll, uint8_t *bwt, uint64_t *term_pos, unsigned char *ws) {
  b.packed = packed;
  b.offsets = offsets;
  b.n = n;
  b.nb = nb;
  b.maxlen = maxlen;
  b.ncoll = ncoll;
  b.bwt = bwt;
  b.term_pos = term_pos;
  b.Lo = make_layout(n, nb, ncoll);
  b.B = buffers_of(ws, b.Lo);
  b.tu = g_tuning;
  b.rmax = maxlen / W + 1;
  b.tile_len = b.tu.tile_len();
  uint32_t *c = b.B.counters;
  b.Ls = Lists{b.B.big_next, c + C_NBIG, (uint32_t)b.Lo.cap_big, b.B.chunks, (unsigned long long *)(c + C_NCHUNK),
               (uint32_t)b.Lo.cap_chunks, b.B.finals, c + C_NFINAL, (uint32_t)b.Lo.cap_finals, c + C_STATUS, b.rmax,
               b.B.stats, b.tu.chunk(), b.tile_len};
  b.coll_reads.assign(coll_reads, coll_reads + ncoll + 1);
}

// Clears the counters, statistics and read-start bitmap, validates the
// offsets and marks the read starts.  With check_bases the collection bases
// are compared with the planned ones (staged in the scan-group area).
int enqueue_prep(const Build &b, const uint64_t *coll_reads_src, const uint64_t *bases_src, PhaseTimer &T,
                 hipStream_t st) {
  const Buffers &B = b.B;
  uint32_t *sbits = B.tile_hist;  // the tile histograms are not used before level 1
  const uint64_t n_sbits = b.nb / 32 + 4;
  if (4 * n_sbits > 4 * 256 * b.Lo.max_tiles) return CXBWT_EDEVICE;
  int rc;
  if ((rc = fill_u32(B.counters, C_COUNT, 0, st))) return rc;
  if ((rc = fill_u64((uint64_t *)B.stats, STAT_WORDS, 0, st))) return rc;
  if ((rc = fill_u32(sbits, n_sbits, 0, st))) return rc;
  CX_CHECK(hipMemcpyAsync(B.coll_reads, coll_reads_src, 8 * ((uint64_t)b.ncoll + 1), hipMemcpyHostToDevice, st));
  T.begin();
  k_prep<<<grid_for(b.n, 256), 256, 0, st>>>(b.packed, b.offsets, b.n, b.nb, b.maxlen, B.coll_reads, b.ncoll, sbits,
                                            b.bwt, b.term_pos, B.counters + C_STATUS);
  CX_LAUNCHED();
  T.end(PH_PREP);
  k_coll_bases<<<grid_for((uint64_t)b.ncoll + 1, 256), 256, 0, st>>>(b.offsets, B.coll_reads, b.ncoll,
                                                                     B.coll_bases);
  CX_LAUNCHED();
  if (bases_src) {
    uint64_t *want = (uint64_t *)B.gsum;
    CX_CHECK(hipMemcpyAsync(want, bases_src, 8 * ((uint64_t)b.ncoll + 1), hipMemcpyHostToDevice, st));
    k_check_bases<<<grid_for((uint64_t)b.ncoll + 1, 256), 256, 0, st>>>(B.coll_bases, want, b.ncoll + 1,
                                                                        B.counters + C_STATUS);
    CX_LAUNCHED();
  }
  return CXBWT_OK;
}

// Text records and the read-start ranks: they need the read-start bitmap
// only, so they are enqueued before the host waits for the level-1 plan.
int enqueue_records(const Build &b, PhaseTimer &T, hipStream_t st) {
  const Buffers &B = b.B;
  const Layout &Lo = b.Lo;
  if (b.nb == 0) return CXBWT_OK;
  uint32_t *sbits = B.tile_hist;
  T.begin();
  k_text_records<<<grid_for(Lo.n_rec, 256), 256, 0, st>>>(b.packed, cxbwt_packed_words(b.nb), sbits, B.text,
                                                           Lo.n_rec);
  CX_LAUNCHED();
  k_rank_count<<<(unsigned)Lo.n_rank_blocks, BLOCK, 0, st>>>(sbits, Lo.n_rank_words, B.rank_blocks);
  CX_LAUNCHED();
  k_rank_top<<<1, BLOCK, 0, st>>>(B.rank_blocks, (uint32_t)Lo.n_rank_blocks);
  CX_LAUNCHED();
  k_rank_words<<<(unsigned)Lo.n_rank_blocks, BLOCK, 0, st>>>(sbits, Lo.n_rank_words, B.rank_blocks, B.srank,
                                                              Lo.n_rec);
  CX_LAUNCHED();
  T.end(PH_PREP);
  return CXBWT_OK;
}

// Reads the collection bases back and plans level 1: the collections above
// one chunk are its segments, the others one unsplit chunk each.
int plan_level1(Build &b, PhaseTimer &T, hipStream_t st) {
  uint32_t hc[C_COUNT];
  b.cbase.assign((size_t)b.ncoll + 1, 0);
  CX_CHECK(hipMemcpyAsync(hc, b.B.counters, sizeof(hc), hipMemcpyDeviceToHost, st));
  CX_CHECK(hipMemcpyAsync(b.cbase.data(), b.B.coll_bases, 8 * ((uint64_t)b.ncoll + 1), hipMemcpyDeviceToHost, st));
  CX_CHECK(hipStreamSynchronize(st));
  T.collect();
  if (hc[C_STATUS] & (ST_BAD_OFFSETS | ST_TOO_LONG)) return CXBWT_EDATA;
  // offsets are valid, so the collection bases are non-decreasing and end at nb
  b.cm.assign(b.ncoll, CollMap{});
  b.big.clear();
  b.small.clear();
  for (uint32_t c = 0; c < b.ncoll; ++c) {
    const uint64_t nc = b.coll_reads[c + 1] - b.coll_reads[c];
    const uint64_t bc = b.cbase[c + 1] - b.cbase[c];
    b.cm[c].out_shift = b.coll_reads[c + 1];
    b.cm[c].row_shift = (int64_t)nc - (int64_t)b.cbase[c];
    if (bc > (uint64_t)b.tu.chunk()) b.big.push_back(Seg{(uint32_t)b.cbase[c], (uint32_t)bc, 0, 0, 0, 0, 0, c});
    else if (bc > 0) b.small.push_back(Seg{(uint32_t)b.cbase[c], (uint32_t)bc, 0, 0, 0, 0, 1, c});
  }
  return CXBWT_OK;
}

// Host sources of the level-1 copies: the segment lists with their tile
// and group prefixes.  An eager build points them at vectors; a captured
// build at pinned memory that lives as long as its graph.
struct SegSrc {
  const Seg *segs = nullptr;
  const uint32_t *tprefix = nullptr, *gprefix = nullptr;
  uint32_t ns = 0, ntiles = 0, ngroups = 0;
};
struct Level1Src {
  const CollMap *cm = nullptr;
  SegSrc big, small;
  const uint32_t *nsmall = nullptr;
};

void seg_prefixes(const std::vector<Seg> &segs, uint32_t tile_len, std::vector<uint32_t> &tp,
                  std::vector<uint32_t> &gp) {
  const size_t ns = segs.size();
  tp.assign(ns + 1, 0);
  gp.assign(ns + 1, 0);
  for (size_t i = 0; i < ns; ++i) {
    const uint32_t nt = (uint32_t)ceil_div(segs[i].len, tile_len);
    tp[i + 1] = tp[i] + nt;
    gp[i + 1] = gp[i] + (uint32_t)ceil_div(nt, GROUP_TILES);
  }
}

int upload_src(const Buffers &B, const Layout &Lo, const SegSrc &s, hipStream_t st) {
  if (s.ns > Lo.seg_slots || s.ntiles > Lo.max_tiles || s.ngroups > Lo.max_groups) return CXBWT_EDEVICE;
  CX_CHECK(hipMemcpyAsync(B.segs, s.segs, sizeof(Seg) * s.ns, hipMemcpyHostToDevice, st));
  CX_CHECK(hipMemcpyAsync(B.tile_prefix, s.tprefix, 4 * ((uint64_t)s.ns + 1), hipMemcpyHostToDevice, st));
  CX_CHECK(hipMemcpyAsync(B.group_prefix, s.gprefix, 4 * ((uint64_t)s.ns + 1), hipMemcpyHostToDevice, st));
  return CXBWT_OK;
}

// The final groups of the current level, with their count on the device.
int finish_finals_dev(const Build &b, hipStream_t st, unsigned emit_grid = PG_EMIT) {
  const Buffers &B = b.B;
  int rc;
  if ((rc = prefix_list(B, B.finals, (uint32_t)b.Lo.cap_finals, b.tile_len, nullptr, B.tile_prefix, nullptr, st,
                        B.counters + C_NFINAL)))
    return rc;
  k_emit_final<true><<<emit_grid, BLOCK, 0, st>>>(B.finals, B.tile_prefix, 0, B.counters + C_NFINAL, b.tile_len, B.keys0,
                                          B.keys1, B.hdl0, B.hdl1, B.text, B.srank, B.cmap, b.bwt, B.start_row);
  CX_LAUNCHED();
  return CXBWT_OK;
}

// Levels 2.. on the host's schedule: every segment of a level is split by
// one digit.  A level that fits the per-segment and per-tile scratch runs
// as one batch whose segment list is prepared on the device; a larger one
// is cut into batches on the host.  acc is what the previous level handed
// on, nbig its segment count.
int run_levels(const Build &b, LevelOut acc, uint32_t nbig, PhaseTimer &T, hipStream_t st) {
  const Buffers &B = b.B;
  const Layout &Lo = b.Lo;
  uint32_t *counters = B.counters;
  std::vector<Seg> big;
  std::vector<uint32_t> tprefix, gprefix;
  uint32_t ntiles = 0, ngroups = 0;
  LevelOut o{};
  int rc;
  while (nbig) {
    if (nbig > Lo.cap_big) return CXBWT_EDEVICE;
    g_stats.levels++;
    g_stats.big_segments += nbig;
    g_stats.level_suffixes += acc.next_len;
    g_stats.regathered += acc.next_regather;
    g_stats.max_window = std::max<uint32_t>(g_stats.max_window, (uint32_t)acc.next_maxr);
    const uint64_t lt = acc.next_tiles, lg = acc.next_groups;
    acc = LevelOut{};
    if ((rc = fill_u32(counters + C_NBIG, 1, 0, st))) return rc;
    if (nbig <= Lo.seg_slots && lt <= Lo.max_tiles && lg <= Lo.max_groups) {
      if ((rc = prefix_list(B, B.big_next, nbig, b.tile_len, B.segs, B.tile_prefix, B.group_prefix, st))) return rc;
      if ((rc = run_level_batch(B, Lo, b.tu, b.Ls, b.nb, b.rmax, b.bwt, nbig, (uint32_t)lt, (uint32_t)lg, o, T,
                                st)))
        return rc;
      record_shape(g_stats.levels - 1, LevelShape{nbig, (uint32_t)lt, (uint32_t)lg, o.n_chunks, o.n_finals,
                                                  (uint32_t)o.final_tiles});
      acc = o;
    } else {
      big.resize(nbig);
      CX_CHECK(hipMemcpyAsync(big.data(), B.big_next, sizeof(Seg) * nbig, hipMemcpyDeviceToHost, st));
      CX_CHECK(hipStreamSynchronize(st));
      for (size_t b0 = 0; b0 < big.size();) {
        const size_t b1 = batch_end(big, b0, Lo, b.tile_len);
        const std::vector<Seg> part(big.begin() + b0, big.begin() + b1);
        if ((rc = upload_segments(B, Lo, part, b.tile_len, tprefix, gprefix, ntiles, ngroups, st))) return rc;
        if ((rc = run_level_batch(B, Lo, b.tu, b.Ls, b.nb, b.rmax, b.bwt, (uint32_t)part.size(), ntiles, ngroups, o,
                                  T, st)))
          return rc;
        record_shape(g_stats.levels - 1, LevelShape{(uint32_t)part.size(), ntiles, ngroups, o.n_chunks, o.n_finals,
                                                    (uint32_t)o.final_tiles});
        acc.next_len += o.next_len;
        acc.next_regather += o.next_regather;
        acc.next_maxr = std::max(acc.next_maxr, o.next_maxr);
        acc.next_tiles += o.next_tiles;
        acc.next_groups += o.next_groups;
        b0 = b1;
      }
    }
    nbig = o.n_big;
  }
  return CXBWT_OK;
}

// Text records, read-end ranks, the collections that fit one chunk, and
// level 1.  Then either (device_levels = 0) the host schedules levels 2..
// with a counter readback per level, or the next device_levels levels are
// enqueued with their sizes read on the device (no host wait: the whole
// sequence can be captured), followed by a last step that flags segments
// left over.  Ends with term_pos.
int enqueue_body(const Build &b, const Level1Src &src, uint32_t device_levels, PhaseTimer &T, hipStream_t st,
                 const std::vector<LevelShape> *shapes = nullptr) {
  const Buffers &B = b.B;
  const Layout &Lo = b.Lo;
  uint32_t *counters = B.counters;
  const uint64_t nb = b.nb;
  int rc;
  if (b.ncoll) CX_CHECK(hipMemcpyAsync(B.cmap, src.cm, sizeof(CollMap) * b.ncoll, hipMemcpyHostToDevice, st));
  if (nb == 0) return CXBWT_OK;

  // collections that fit one chunk: keys in read order, one unsplit chunk each
  if (src.small.ns) {
    if ((rc = upload_src(B, Lo, src.small, st))) return rc;
    T.begin();
    k_gen<<<src.small.ntiles, BLOCK, 0, st>>>(B.segs, B.tile_prefix, src.small.ns, b.tile_len, B.text, nb, B.keys0,
                                              B.hdl0);
    CX_LAUNCHED();
    T.end(PH_GEN);
    CX_CHECK(hipMemcpyAsync(B.chunks, src.small.segs, sizeof(Seg) * src.small.ns, hipMemcpyHostToDevice, st));
    if (!src.big.ns) {
      if ((rc = finish_level(B, Lo, b.tu, nb, b.rmax, b.bwt, src.small.ns, 0, 0, 0, T, st))) return rc;
    } else {
      // level 1 appends its chunks after these
      CX_CHECK(hipMemcpyAsync(counters + C_NCHUNK, src.nsmall, 4, hipMemcpyHostToDevice, st));
    }
  }
  if (src.big.ns) {
    // level 1: keys computed from the 2-bit reads, counted, recomputed, scattered
    const uint32_t ns = src.big.ns, ntiles = src.big.ntiles, ngroups = src.big.ngroups;
    if ((rc = upload_src(B, Lo, src.big, st))) return rc;
    T.begin();
    if (b.tu.tile_items == 16)
      k_gen_hist<2><<<ntiles, BLOCK, 0, st>>>(B.segs, B.tile_prefix, ns, b.tile_len, B.text, nb, B.tile_hist);
    else
      k_gen_hist<1><<<ntiles, BLOCK, 0, st>>>(B.segs, B.tile_prefix, ns, b.tile_len, B.text, nb, B.tile_hist);
    CX_LAUNCHED();
    T.end(PH_GEN);
    T.begin();
    k_group_scan<false><<<ngroups, BLOCK, 0, st>>>(B.tile_prefix, B.group_prefix, ns, nullptr, B.tile_hist, B.gsum);
    CX_LAUNCHED();
    launch_level_scan(B, ns, ngroups, b.Ls, 1, st);
    CX_LAUNCHED();
    T.end(PH_SCAN);
    T.begin();
#define CX_GEN_SCATTER(TI, NW)                                                                                    \
  k_gen_scatter<TI, NW><<<ntiles, 64 * NW, 0, st>>>(B.segs, B.tile_prefix, B.group_prefix, ns, B.text, nb,         \
                                                    B.tile_hist, B.gsum, B.keys1, B.hdl1)
    if (b.tu.tile_items == 16) CX_GEN_SCATTER(8, 8);
    else if (b.tu.tile_items == 8) CX_GEN_SCATTER(8, 4);
    else CX_GEN_SCATTER(6, 4);
#undef CX_GEN_SCATTER
    CX_LAUNCHED();
    T.end(PH_SCATTER);
    if (device_levels == 0) {
      LevelOut o{};
      if ((rc = read_level(B, o, T, st))) return rc;
      record_shape(0, LevelShape{ns, ntiles, ngroups, o.n_chunks, o.n_finals, (uint32_t)o.final_tiles});
      if ((rc = finish_level(B, Lo, b.tu, nb, b.rmax, b.bwt, o.n_chunks, o.n_finals, o.final_tiles, o.final_len, T,
                             st)))
        return rc;
      if ((rc = run_levels(b, o, o.n_big, T, st))) return rc;
    } else {
      const uint32_t *ncur = counters + C_NCUR;
      const LevelShape none;
      auto seen = [&](uint32_t lv) -> const LevelShape & {
        return shapes && lv < shapes->size() ? (*shapes)[lv] : none;
      };
      for (uint32_t lv = 0;; ++lv) {
        // the level just scanned: fold, finish its chunks and final groups
        k_level_fold<<<1, 64, 0, st>>>(B.stats, (unsigned long long *)(counters + C_FOLD), counters + C_FLAGS);
        CX_LAUNCHED();
        if ((rc = launch_local(B, b.tu, nb, b.rmax, b.bwt, (uint32_t)Lo.cap_chunks, counters + C_NCHUNK, st,
                               grid_from(seen(lv).nchunks, 0))))
          return rc;
        if ((rc = finish_finals_dev(b, st, grid_from(seen(lv).ftiles, PG_EMIT)))) return rc;
        const int last = lv == device_levels - 1;
        k_level_step<<<1, 64, 0, st>>>(counters, Lo.seg_slots, Lo.max_tiles, Lo.max_groups, last);
        CX_LAUNCHED();
        if (last) break;
        // the next level, sized on the device
        if ((rc = prefix_list(B, B.big_next, (uint32_t)Lo.seg_slots, b.tile_len, B.segs, B.tile_prefix,
                              B.group_prefix, st, ncur)))
          return rc;
        k_fill_seg<<<PG_FILL, 256, 0, st>>>(B.seg_or, B.seg_and, ncur);
        CX_LAUNCHED();
        if ((rc = launch_level_kernels(B, b.tu, b.Ls, nb, 0, 0, 0, ncur, T, st, &seen(lv + 1)))) return rc;
      }
    }
  }
  T.begin();
  k_term<<<grid_for(b.n, 256), 256, 0, st>>>(b.offsets, b.n, b.nb, B.text, B.srank, B.start_row, b.term_pos);
  CX_LAUNCHED();
  T.end(PH_FINAL);
  return CXBWT_OK;
}

// Statistics counters of the build, and the device status.
int read_totals(const Build &b, PhaseTimer &T, hipStream_t st, uint32_t (&hc)[C_COUNT]) {
  std::vector<uint64_t> hs(STAT_WORDS);
  CX_CHECK(hipMemcpyAsync(hc, b.B.counters, sizeof(hc), hipMemcpyDeviceToHost, st));
  CX_CHECK(hipMemcpyAsync(hs.data(), b.B.stats, 8 * STAT_WORDS, hipMemcpyDeviceToHost, st));
  CX_CHECK(hipStreamSynchronize(st));
  T.collect();
  for (int i = 0; i < STAT_SPREAD; ++i) {
    g_stats.window_fetches += hs[K_FETCHES * STAT_KIND + i * STAT_STRIDE];
    g_stats.scattered_suffixes += hs[K_SCATTERED * STAT_KIND + i * STAT_STRIDE];
  }
  return CXBWT_OK;
}

// Level-1 sources taken from the plan's vectors (an eager build).
struct Level1Vectors {
  std::vector<uint32_t> btp, bgp, stp, sgp;
  uint32_t nsmall = 0;
  Level1Src src;
  void make(const Build &b) {
    seg_prefixes(b.big, b.tile_len, btp, bgp);
    seg_prefixes(b.small, b.tile_len, stp, sgp);
    nsmall = (uint32_t)b.small.size();
    src.cm = b.cm.data();
    src.big = SegSrc{b.big.data(), btp.data(), bgp.data(), (uint32_t)b.big.size(), btp.back(), bgp.back()};
    src.small = SegSrc{b.small.data(), stp.data(), sgp.data(), nsmall, stp.back(), sgp.back()};
    src.nsmall = &nsmall;
  }
};

void level1_stats(const Build &b) {
  g_stats.chunk_suffixes = b.nb;
  if (!b.big.empty()) {
    g_stats.levels = 1;
    g_stats.big_segments = b.big.size();
    for (const Seg &g : b.big) g_stats.level_suffixes += g.len;
  }
}

// The whole build for ncoll collections laid end to end (a single build is
// one collection).  coll_reads (host) holds ncoll + 1 read boundaries.
int run_build(const uint64_t *packed, const uint64_t *offsets, uint64_t n, uint64_t nb, uint32_t maxlen,
              const uint64_t *coll_reads, uint32_t ncoll, uint8_t *bwt, uint64_t *term_pos, unsigned char *ws,
              hipStream_t st, bool allow_timing = true) {
  g_stats = cxbwt_stats{};
  PhaseTimer T{st, allow_timing && g_timing != 0, {}};
  Build b;
  build_init(b, packed, offsets, n, nb, maxlen, coll_reads, ncoll, bwt, term_pos, ws);
  int rc;
  if ((rc = enqueue_prep(b, b.coll_reads.data(), nullptr, T, st))) return rc;
  if ((rc = enqueue_records(b, T, st))) return rc;
  if ((rc = plan_level1(b, T, st))) return rc;
  Level1Vectors v;
  v.make(b);
  level1_stats(b);
  if ((rc = enqueue_body(b, v.src, 0, T, st))) return rc;
  uint32_t hc[C_COUNT];
  if ((rc = read_totals(b, T, st, hc))) return rc;
  if (hc[C_STATUS]) return CXBWT_EDEVICE;
  return CXBWT_OK;
}

// A build captured once in a hipGraph for fixed sizes and buffers, replayed
// on new contents of the same buffers.
struct GraphPlan {
  Build b;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned char *pinned = nullptr;  // host sources of the captured copies
  uint32_t levels = 0;              // levels scheduled on the device, level 1 included
  cxbwt_stats base{};               // statistics of level 1 (known on the host)
  std::vector<LevelShape> shapes;   // per-level counts of the eager build made at creation
  ~GraphPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (pinned) (void)hipHostFree(pinned);
  }
};

int graph_capture(GraphPlan &P, hipStream_t st) {
  Build &b = P.b;
  PhaseTimer T{st, false, {}};
  // eager build: validates the offsets, learns the collection bases and
  // records every level's counts, which size the captured launches
  int rc;
  if ((rc = enqueue_prep(b, b.coll_reads.data(), nullptr, T, st))) return rc;
  if ((rc = enqueue_records(b, T, st))) return rc;
  if ((rc = plan_level1(b, T, st))) return rc;
  Level1Vectors v;
  v.make(b);
  g_stats = cxbwt_stats{};
  level1_stats(b);
  P.base = g_stats;
  P.shapes.clear();
  g_shapes = &P.shapes;
  rc = enqueue_body(b, v.src, 0, T, st);
  g_shapes = nullptr;
  uint32_t hc[C_COUNT];
  if (!rc) rc = read_totals(b, T, st, hc);
  if (rc) return rc;
  if (hc[C_STATUS]) return CXBWT_EDEVICE;
  // pinned copies of everything the captured copies read
  const size_t nc1 = (size_t)b.ncoll + 1;
  const size_t nbg = b.big.size(), nsm = b.small.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t o_cr = take(8 * nc1), o_cb = take(8 * nc1), o_cm = take(sizeof(CollMap) * b.ncoll),
               o_bs = take(sizeof(Seg) * nbg), o_btp = take(4 * (nbg + 1)), o_bgp = take(4 * (nbg + 1)),
               o_ss = take(sizeof(Seg) * nsm), o_stp = take(4 * (nsm + 1)), o_sgp = take(4 * (nsm + 1)),
               o_ns = take(4);
  CX_CHECK(hipHostMalloc((void **)&P.pinned, off, hipHostMallocDefault));
  unsigned char *h = P.pinned;
  memcpy(h + o_cr, b.coll_reads.data(), 8 * nc1);
  memcpy(h + o_cb, b.cbase.data(), 8 * nc1);
  if (b.ncoll) memcpy(h + o_cm, b.cm.data(), sizeof(CollMap) * b.ncoll);
  if (nbg) memcpy(h + o_bs, b.big.data(), sizeof(Seg) * nbg);
  memcpy(h + o_btp, v.btp.data(), 4 * (nbg + 1));
  memcpy(h + o_bgp, v.bgp.data(), 4 * (nbg + 1));
  if (nsm) memcpy(h + o_ss, b.small.data(), sizeof(Seg) * nsm);
  memcpy(h + o_stp, v.stp.data(), 4 * (nsm + 1));
  memcpy(h + o_sgp, v.sgp.data(), 4 * (nsm + 1));
  memcpy(h + o_ns, &v.nsmall, 4);
  Level1Src src;
  src.cm = (const CollMap *)(h + o_cm);
  src.big = SegSrc{(const Seg *)(h + o_bs), (const uint32_t *)(h + o_btp), (const uint32_t *)(h + o_bgp),
                   (uint32_t)nbg, v.btp.back(), v.bgp.back()};
  src.small = SegSrc{(const Seg *)(h + o_ss), (const uint32_t *)(h + o_stp), (const uint32_t *)(h + o_sgp),
                     (uint32_t)nsm, v.stp.back(), v.sgp.back()};
  src.nsmall = (const uint32_t *)(h + o_ns);
  // capture: every size below is fixed now or read on the device
  CX_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  rc = enqueue_prep(b, (const uint64_t *)(h + o_cr), (const uint64_t *)(h + o_cb), T, st);
  if (!rc) rc = enqueue_records(b, T, st);
  if (!rc) rc = enqueue_body(b, src, P.levels ? P.levels : 1, T, st, &P.shapes);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (ec != hipSuccess || !g) return CXBWT_EDEVICE;
  P.graph = g;
  CX_CHECK(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
  return CXBWT_OK;
}

// After a replay: status, statistics, and the levels left to the host.
int graph_finish(GraphPlan &P, hipStream_t st) {
  Build &b = P.b;
  PhaseTimer T{st, false, {}};
  g_stats = P.base;
  uint32_t hc[C_COUNT];
  int rc;
  if ((rc = read_totals(b, T, st, hc))) return rc;
  if (hc[C_STATUS] & (ST_BAD_OFFSETS | ST_TOO_LONG)) return CXBWT_EDATA;
  if (hc[C_STATUS] & ST_PLAN_MISMATCH) return CXBWT_EINVAL;
  if (hc[C_STATUS]) return CXBWT_EDEVICE;
  uint64_t g[G_COUNT], f[K_LEVEL_KINDS];
  memcpy(g, hc + C_CUM, sizeof(g));
  memcpy(f, hc + C_FOLD, sizeof(f));
  g_stats.levels += (uint32_t)g[G_LEVELS];
  g_stats.big_segments += g[G_BIGSEG];
  g_stats.level_suffixes += g[G_LEVSUF];
  g_stats.regathered += g[G_REGATH];
  g_stats.max_window = std::max<uint32_t>(g_stats.max_window, (uint32_t)g[G_MAXWIN]);
  g_stats.chunks += g[G_CHUNKS];
  g_stats.final_big += g[G_FINALS];
  g_stats.chunk_suffixes -= g[G_FINLEN];
  g_stats.level_batches += (uint32_t)g[G_BATCHES];
  if (!(hc[C_FLAGS] & (FL_STALLED | FL_INCOMPLETE))) return CXBWT_OK;
  // the device schedule did not cover the build: the host finishes it
  LevelOut acc{};
  acc.next_len = f[K_NEXT_LEN - K_LEVEL_FIRST];
  acc.next_regather = f[K_NEXT_REGATHER - K_LEVEL_FIRST];
  acc.next_maxr = f[K_NEXT_MAXR - K_LEVEL_FIRST];
  acc.next_tiles = f[K_NEXT_TILES - K_LEVEL_FIRST];
  acc.next_groups = f[K_NEXT_GROUPS - K_LEVEL_FIRST];
  if ((rc = run_levels(b, acc, hc[C_NBIG], T, st))) return rc;
  k_term<<<grid_for(b.n, 256), 256, 0, st>>>(b.offsets, b.n, b.nb, b.B.text, b.B.srank, b.B.start_row,
                                              b.term_pos);
  CX_LAUNCHED();
  // the statistics block still holds the replay's counts: take the rest only
  g_stats.window_fetches = 0;
  g_stats.scattered_suffixes = 0;
  if ((rc = read_totals(b, T, st, hc))) return rc;
  if (hc[C_STATUS]) return CXBWT_EDEVICE;
  return CXBWT_OK;
}

}  // namespace

struct cxbwt_graph {
  GraphPlan p;
};

// Workspace of cxbwt_build_noalloc: a fixed array in the code object, one
// copy per device the library runs on, held until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it
// names a stand-in, not device memory): it uses the device address
// hipGetSymbolAddress returns, taken once per device with that device
// current and kept in g_scratch_addr.
static __device__ __align__(256) unsigned char scratch[CXBWT_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_addr[SCRATCH_MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`.
int scratch_address(unsigned char **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES) return CXBWT_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CXBWT_EDEVICE;
    if (((uintptr_t)p & 255u) != 0) return CXBWT_EDEVICE;
    g_scratch_addr[dev] = (unsigned char *)p;
  }
  *out = g_scratch_addr[dev];
  return CXBWT_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

uint64_t cxbwt_packed_words(uint64_t n_bases) { return (n_bases + 31) / 32 + 1; }

int cxbwt_pack(const uint8_t *ascii, uint64_t n_bases, uint64_t *packed, uint32_t *d_status, void *stream) {
  if (n_bases > CXBWT_MAX_BASES) return CXBWT_ERANGE;
  if (!packed || (n_bases && !ascii)) return CXBWT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (d_status) {
    int rc = fill_u32(d_status, 1, 0, st);
    if (rc) return rc;
  }
  const uint64_t nw = cxbwt_packed_words(n_bases);
  k_pack<<<grid_for(nw, 256), 256, 0, st>>>(ascii, n_bases, packed, nw, d_status);
  if (hipGetLastError() != hipSuccess) return CXBWT_EDEVICE;
  return CXBWT_OK;
}

size_t cxbwt_workspace_bytes(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len) {
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return 0;
  return (size_t)make_layout(n_reads, n_bases, 1).total;
}

size_t cxbwt_batch_workspace_bytes(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len, uint32_t n_coll) {
  if (!sizes_ok(n_reads, n_bases, max_read_len) || n_coll == 0 || n_coll > n_reads) return 0;
  return (size_t)make_layout(n_reads, n_bases, n_coll).total;
}

int cxbwt_build(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                uint32_t max_read_len, uint8_t *bwt, uint64_t *term_pos, void *workspace, size_t workspace_bytes,
                void *stream) {
  if (!packed || !offsets || !bwt || !term_pos || !workspace || n_reads == 0) return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (workspace_bytes < cxbwt_workspace_bytes(n_reads, n_bases, max_read_len)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  const uint64_t one[2] = {0, n_reads};
  return run_build(packed, offsets, n_reads, n_bases, max_read_len, one, 1, bwt, term_pos, (unsigned char *)workspace,
                   (hipStream_t)stream);
}

int cxbwt_build_noalloc(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                        uint32_t max_read_len, uint8_t *bwt, uint64_t *term_pos, void *stream) {
  if (!packed || !offsets || !bwt || !term_pos || n_reads == 0) return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (cxbwt_workspace_bytes(n_reads, n_bases, max_read_len) > CXBWT_NOALLOC_WORKSPACE_BYTES) return CXBWT_ESCRATCH;
  unsigned char *ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  const uint64_t one[2] = {0, n_reads};
  // no kernel timing here: it would create HIP events
  return run_build(packed, offsets, n_reads, n_bases, max_read_len, one, 1, bwt, term_pos, ws, (hipStream_t)stream,
                   false);
}

int cxbwt_build_batch(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                      uint32_t max_read_len, const uint64_t *coll_reads, uint32_t n_coll, uint8_t *bwt,
                      uint64_t *term_pos, void *workspace, size_t workspace_bytes, void *stream) {
  if (!packed || !offsets || !bwt || !term_pos || !workspace || !coll_reads || n_reads == 0 || n_coll == 0)
    return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (n_coll > n_reads) return CXBWT_EINVAL;
  if (coll_reads[0] != 0 || coll_reads[n_coll] != n_reads) return CXBWT_EINVAL;
  for (uint32_t c = 0; c < n_coll; ++c)
    if (coll_reads[c + 1] <= coll_reads[c]) return CXBWT_EINVAL;  // every collection holds a read
  if (workspace_bytes < cxbwt_batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  return run_build(packed, offsets, n_reads, n_bases, max_read_len, coll_reads, n_coll, bwt, term_pos,
                   (unsigned char *)workspace, (hipStream_t)stream);
}

int cxbwt_graph_create(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                       uint32_t max_read_len, const uint64_t *coll_reads, uint32_t n_coll, uint8_t *bwt,
                       uint64_t *term_pos, void *workspace, size_t workspace_bytes, uint32_t levels, void *stream,
                       cxbwt_graph **out) {
  if (!out) return CXBWT_EINVAL;
  *out = nullptr;
  if (!packed || !offsets || !bwt || !term_pos || !workspace || n_reads == 0 || n_coll == 0) return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  const uint64_t one[2] = {0, n_reads};
  if (!coll_reads) {
    if (n_coll != 1) return CXBWT_EINVAL;
    coll_reads = one;
  }
  if (n_coll > n_reads || coll_reads[0] != 0 || coll_reads[n_coll] != n_reads) return CXBWT_EINVAL;
  for (uint32_t c = 0; c < n_coll; ++c)
    if (coll_reads[c + 1] <= coll_reads[c]) return CXBWT_EINVAL;
  if (workspace_bytes < cxbwt_batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  cxbwt_graph *g = new (std::nothrow) cxbwt_graph;
  if (!g) return CXBWT_ENOMEM;
  build_init(g->p.b, packed, offsets, n_reads, n_bases, max_read_len, coll_reads, n_coll, bwt, term_pos,
             (unsigned char *)workspace);
  g->p.levels = levels ? levels : 8 * g->p.b.rmax + 2;
  // the eager pass runs on the caller's stream; the capture on a stream of
  // its own (a capture needs a non-default stream)
  hipStream_t cs = nullptr;
  int rc = CXBWT_OK;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = CXBWT_EDEVICE;
  if (!rc && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = CXBWT_EDEVICE;
  if (!rc) rc = graph_capture(g->p, cs);
  if (cs) (void)hipStreamDestroy(cs);
  if (rc) {
    delete g;
    return rc;
  }
  *out = g;
  return CXBWT_OK;
}

int cxbwt_graph_launch(cxbwt_graph *g, void *stream) {
  if (!g || !g->p.exec) return CXBWT_EINVAL;
  return hipGraphLaunch(g->p.exec, (hipStream_t)stream) == hipSuccess ? CXBWT_OK : CXBWT_EDEVICE;
}

int cxbwt_graph_finish(cxbwt_graph *g, void *stream) {
  if (!g || !g->p.exec) return CXBWT_EINVAL;
  return graph_finish(g->p, (hipStream_t)stream);
}

void cxbwt_graph_destroy(cxbwt_graph *g) { delete g; }

int cxbwt_last_stats(cxbwt_stats *out) {
  if (!out) return CXBWT_EINVAL;
  *out = g_stats;
  return CXBWT_OK;
}

int cxbwt_set_tuning(uint32_t tile_items, uint32_t chunk_items) {
  if (!tuning_ok(tile_items, chunk_items)) return CXBWT_EINVAL;
  g_tuning = Tuning{tile_items, chunk_items};
  return CXBWT_OK;
}

int cxbwt_get_tuning(uint32_t *tile_items, uint32_t *chunk_items) {
  if (!tile_items || !chunk_items) return CXBWT_EINVAL;
  *tile_items = g_tuning.tile_items;
  *chunk_items = g_tuning.chunk_items;
  return CXBWT_OK;
}

int cxbwt_set_timing(int enable) {
  const int prev = g_timing;
  g_timing = enable ? 1 : 0;
  return prev;
}

const char *cxbwt_status_str(int status) {
  switch (status) {
    case CXBWT_OK: return "ok";
    case CXBWT_EINVAL: return "invalid argument (null pointer or inconsistent sizes)";
    case CXBWT_ERANGE: return "size out of the supported range";
    case CXBWT_ENOMEM: return "workspace smaller than cxbwt_workspace_bytes()";
    case CXBWT_EDEVICE: return "HIP launch/runtime failure or internal device check failed";
    case CXBWT_EDATA: return "invalid input data found on the device (offsets, read length or bases)";
    case CXBWT_ESCRATCH:
      return "input needs more workspace than cxbwt_build_noalloc's fixed device array holds "
             "(CXBWT_NOALLOC_WORKSPACE_BYTES); use cxbwt_build with a caller workspace";
    default: return "unknown status";
  }
}

}  // extern "C"
