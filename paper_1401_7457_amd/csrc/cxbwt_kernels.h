// cxbwt_kernels.h -- the device side of cxbwt.hip: data records and constants
// shared with the host code, and every kernel of the build.  Included once,
// by cxbwt.hip; kept apart so that the kernel sources can be identified
// (hashed) without the host code that sequences them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// Base position of the suffix a 32-bit handle names: the handle itself, or,
// in a build in ranges with wide positions (more bases than 32 bits count),
// an index into the range's table of 64-bit positions.
__device__ __forceinline__ uint64_t position_of(const uint64_t *__restrict__ pos64, uint32_t h) {
  return pos64 ? pos64[h] : (uint64_t)h;
}

// Writes the BWT row of a sorted suffix; an offset-0 suffix also records its
// row under its read's rank among the non-empty reads (k_term turns those
// into term_pos).
__device__ __forceinline__ void emit_row(uint64_t j, const CollMap &cm, uint64_t key, uint32_t h,
                                         const uint64_t *__restrict__ pos64, const TextRec *__restrict__ text,
                                         const uint32_t *__restrict__ srank, uint8_t *__restrict__ bwt,
                                         uint64_t *__restrict__ start_row) {
  const uint32_t pv = (uint32_t)key & 7u;
  const uint32_t lut = 'A' | ('C' << 8) | ('G' << 16) | ('T' << 24);
  bwt[j + cm.out_shift] = pv == 4 ? (uint8_t)'$' : (uint8_t)((lut >> (8 * pv)) & 0xFFu);
  if (pv == 4) start_row[start_rank(text, srank, position_of(pos64, h))] = (uint64_t)((int64_t)j + cm.row_shift);
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
  // the end of the text ends every window, also when offsets are invalid
  // (the levels of a device-scheduled build still run over [0, nb))
  if (i == n - 1) atomicOr(&sbits[nb >> 5], 1u << (nb & 31));
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
  // every record load of a sub-tile is issued before its first key is formed
  // (an item past the tile reads the last one's record, t1 > t0)
#pragma unroll
  for (int sub = 0; sub < SUBT; ++sub) {
    const uint64_t u0 = t0 + (uint64_t)sub * BLOCK * MAX_TILE_ITEMS;
    TextRec tr[MAX_TILE_ITEMS];
#pragma unroll
    for (int i = 0; i < MAX_TILE_ITEMS; ++i) {
      const uint64_t p = u0 + (uint64_t)i * BLOCK + threadIdx.x;
      tr[i] = text[(p < t1 ? p : t1 - 1) >> 4];
    }
#pragma unroll
    for (int i = 0; i < MAX_TILE_ITEMS; ++i) {
      const uint64_t p = u0 + (uint64_t)i * BLOCK + threadIdx.x;
      if (p < t1) atomicAdd(&hist[digit_of(first_key_from(tr[i], nb, p), 0)], 1u);
    }
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
  // the records of every item are loaded before any key is formed (an item
  // past the tile reads the last one's record, m >= 1)
  TextRec tr[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const uint32_t li = item_index<TI>(i);
    tr[i] = text[(t0 + (li < m ? li : m - 1)) >> 4];
  }
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const uint32_t li = item_index<TI>(i);
    if (li < m) {
      kr[i] = first_key_from(tr[i], nb, t0 + li);
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
                                                      const uint64_t *__restrict__ pos64,
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
  // then records) are issued before any result is used; the sub-tiles one
  // after the other (holding both sets of keys at once costs more in
  // occupancy than the second wait)
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
      uint64_t hh[MAX_TILE_ITEMS];
      TextRec tr[MAX_TILE_ITEMS];
#pragma unroll
      for (int i = 0; i < MAX_TILE_ITEMS; ++i)
        if (in[i]) hh[i] = H[u0 + (uint64_t)i * BLOCK + threadIdx.x];
      if (pos64) {
#pragma unroll
        for (int i = 0; i < MAX_TILE_ITEMS; ++i)
          if (in[i]) hh[i] = pos64[hh[i]];
      }
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
  // every load of the tile is issued before any is used (an item past the
  // tile reads the last one, m >= 1, and is then cleared)
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const uint32_t li = item_index<TI>(i);
    const uint64_t at = t0 + (li < m ? li : m - 1);
    kr[i] = Ki[at];
    hr[i] = Hi[at];
  }
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    if (item_index<TI>(i) < m) {
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
                                                      const uint32_t *__restrict__ hdl1, const uint64_t *__restrict__ pos64,
                                                      const TextRec *__restrict__ text,
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
    for (uint64_t j = t0 + threadIdx.x; j < t1; j += BLOCK)
      emit_row(j, cm, K[j], H[j], pos64, text, srank, bwt, start_row);
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
// (about 6.4 KB for 384 suffixes: six one-wave workgroups per SIMD)
template <int LI>
struct LocalSmem {
  static constexpr int CHUNK = LOCAL_WG * LI;
  uint64_t K[CHUNK];  // key of each position
  uint32_t H[CHUNK];  // handle of each position
  union {
    struct {
      uint16_t live[CHUNK];  // live positions, ascending
      // group of each live-list entry; while a sort moves the entries, the
      // entry's new position (each entry's own lane reads the group first)
      uint16_t gr[CHUNK];
      // first live-list entry of each group, then the list length: a kept
      // group has two entries or more
      uint16_t hp[CHUNK / 2 + 1];
    };
    struct {  // while the chunk is split by digits
      uint16_t cnt[256];
      uint16_t dstart[256];
    };
  };
  uint32_t headw[CHUNK / 32];  // bit j % 32 of word j / 32: position j starts a group
};

template <int LI>
__device__ __forceinline__ bool head_at(const LocalSmem<LI> &S, uint32_t j) {
  return (S.headw[j >> 5] >> (j & 31u)) & 1u;
}

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
    const uint64_t peers = wave_match8(dig[i], __ballot(valid));
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

// Live groups of more than BIG_GROUP suffixes are sorted in place by a
// bitonic network instead of the all-pairs ranking, whose cost grows with
// the square of the group.  Equal ordering bits keep the suffixes in handle
// order, which is their order in the group: the first order was read-major
// (handles are base positions, or indices of a position-ordered table) and
// every pass since was stable.  So the network sorts by (ordering bits,
// handle), which are distinct, and gives the same order as a stable rank.
constexpr uint32_t BIG_GROUP = 96;

__device__ __forceinline__ bool rec_after(uint64_t ka, uint32_t ha, uint64_t kb, uint32_t hb) {
  const uint64_t oa = order_bits(ka), ob = order_bits(kb);
  return oa > ob || (oa == ob && ha > hb);
}

// One group of positions [a, a + m): the network for the next power of two
// P >= m with the missing entries taken as larger than all, so that every
// compare-exchange puts the smaller entry first and a pair reaching past the
// group is left as it is.  Each merge of blocks of k starts by comparing
// mirrored entries (i with the entry k - 1 - (i mod k) of its block), then
// halves the distance.
template <int LI>
__device__ __forceinline__ void bitonic_group(LocalSmem<LI> &S, uint32_t a, uint32_t m, uint32_t lane) {
  uint32_t P = 2;
  while (P < m) P <<= 1;
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t d = k >> 1; d > 0; d >>= 1) {
      for (uint32_t q = lane; q < P / 2; q += LOCAL_WG) {
        uint32_t i, l;
        if (d == k >> 1) {  // mirrored pairs of a block of k
          const uint32_t blk = q / d, off = q % d;
          i = blk * k + off;
          l = blk * k + (k - 1 - off);
        } else {
          i = (q / d) * 2 * d + (q % d);
          l = i + d;
        }
        if (l < m) {
          const uint64_t ki = S.K[a + i], kl = S.K[a + l];
          const uint32_t hi = S.H[a + i], hl = S.H[a + l];
          if (rec_after(ki, hi, kl, hl)) {
            S.K[a + i] = kl;
            S.K[a + l] = ki;
            S.H[a + i] = hl;
            S.H[a + l] = hi;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Every live group above BIG_GROUP suffixes, one after another.
template <int LI>
__device__ __forceinline__ void sort_big_groups(LocalSmem<LI> &S, uint32_t ngroups, uint32_t lane) {
  for (uint32_t g0 = 0; g0 < ngroups; g0 += LOCAL_WG) {
    const uint32_t g = g0 + lane;
    const bool big = g < ngroups && (uint32_t)S.hp[g + 1] - S.hp[g] > BIG_GROUP;
    uint64_t todo = __ballot(big);
    while (todo) {
      const uint32_t b = g0 + (uint32_t)__builtin_ctzll(todo);
      todo &= todo - 1;
      const uint32_t x0 = S.hp[b];
      bitonic_group(S, (uint32_t)S.live[x0], (uint32_t)S.hp[b + 1] - x0, lane);
    }
  }
}

// #{t in [a, j) : k_t < below} + #{t in [j, e) : k_t < oj} for the keys
// k_t = p0[STRIDE * t] of one group.  The LDS address is the loop variable,
// tested against a bound three entries early: one add and one compare per
// step of four independent reads.
template <typename T, int STRIDE>
__device__ __forceinline__ uint32_t count_below(const T *p0, uint32_t a, uint32_t j, uint32_t e, T below, T oj) {
  uint32_t c = 0;
  const T *p = p0 + STRIDE * a;
  const T *const pj = p0 + STRIDE * j, *const pe = p0 + STRIDE * e;
  const T *const pj3 = p0 + STRIDE * (j >= 3 ? j - 3 : 0), *const pe3 = p0 + STRIDE * (e >= 3 ? e - 3 : 0);
  for (; p < pj3; p += 4 * STRIDE)
    c += (uint32_t)(p[0] < below) + (uint32_t)(p[STRIDE] < below) + (uint32_t)(p[2 * STRIDE] < below) +
         (uint32_t)(p[3 * STRIDE] < below);
  for (; p < pj; p += STRIDE) c += (uint32_t)(*p < below);
  for (; p < pe3; p += 4 * STRIDE)
    c += (uint32_t)(p[0] < oj) + (uint32_t)(p[STRIDE] < oj) + (uint32_t)(p[2 * STRIDE] < oj) +
         (uint32_t)(p[3 * STRIDE] < oj);
  for (; p < pe; p += STRIDE) c += (uint32_t)(*p < oj);
  return c;
}

// LI suffixes per lane; OCC waves per SIMD the kernel is compiled for;
// PERSIST: a fixed grid loops over a chunk count on the device
template <int LI, int OCC, bool PERSIST>
__global__ __launch_bounds__(LOCAL_WG, OCC) void k_local(
    const Seg *__restrict__ chunks, const uint64_t *__restrict__ keys0, const uint64_t *__restrict__ keys1,
    const uint32_t *__restrict__ hdl0, const uint32_t *__restrict__ hdl1, const uint64_t *__restrict__ pos64,
    const TextRec *__restrict__ text, const uint32_t *__restrict__ srank, const CollMap *__restrict__ cmap,
    uint64_t nb, uint32_t rmax,
    uint8_t *__restrict__ bwt, uint64_t *__restrict__ start_row, uint32_t *status, unsigned long long *fetches,
    uint32_t n_chunks, const uint32_t *__restrict__ dev_nchunks, uint32_t first) {
  __shared__ LocalSmem<LI> S;
  // chunks of up to twice BIG_GROUP suffixes keep the all-pairs ranking for
  // every group (and the registers the network would take)
  constexpr bool SORT_BIG = LI * LOCAL_WG > 2 * (int)BIG_GROUP;
  constexpr bool SPLIT_CHUNKS = LI > 3;
  const uint32_t lane = threadIdx.x;
  const uint64_t le = lanemask_lt() | (1ull << lane);
  // chunks first + blockIdx.x (+ k * gridDim.x when PERSIST) below the count
  if (dev_nchunks) n_chunks = *dev_nchunks;
  uint32_t nfetch = 0;
  for (uint32_t c = first + blockIdx.x; c < n_chunks; c += gridDim.x) {
  if (PERSIST) __syncthreads();  // the previous chunk's LDS reads are done
  const Seg ch = chunks[c];
  const CollMap cm = cmap[ch.coll];  // loaded with the chunk, used at the emit
  const uint32_t m = (uint32_t)ch.len;
  const uint64_t *Kg = ch.buf ? keys1 : keys0;
  const uint32_t *Hg = ch.buf ? hdl1 : hdl0;
  // entry x of a list is handled by lane x % 64 in slot x / 64: neighbouring
  // lanes hold neighbouring positions, which mostly share a group
  // every load of the chunk is issued before the first store to LDS (an
  // entry past the chunk reads the last one, m >= 1)
  {
    uint64_t lk[LI];
    uint32_t lh[LI];
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      const uint32_t j = i * LOCAL_WG + lane;
      const uint64_t at = ch.start + (j < m ? j : m - 1);
      lk[i] = Kg[at];
      lh[i] = Hg[at];
    }
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      const uint32_t j = i * LOCAL_WG + lane;
      if (j < m) {
        S.K[j] = lk[i];
        S.H[j] = lh[i];
      }
    }
  }
  __syncthreads();
  // The chunk is a run of buckets that differ in digit d and agree before
  // it (or, unsplit, in read order, with d = 0).  Two stable splits, by digit
  // d + 1 and then by digit d, leave it ordered by both digits; the groups of
  // equal (d, d + 1) digits are then sorted on their current key, and after
  // that groups are runs of equal keys, refined window by window.
  const int d0 = ch.d;
  // (chunks of up to 3 suffixes a lane hold buckets small enough that the
  // ranking alone is cheaper than the two splits)
  const bool two = SPLIT_CHUNKS && d0 < 7;
  if (two) {
    // a chunk of one bucket (its first and last suffixes share digit d) is
    // ordered by both digits after the first split
    const bool one_bucket = !ch.unsplit && digit_of(S.K[0], d0) == digit_of(S.K[m - 1], d0);
    wave_split(S, m, d0 + 1, lane, le & ~(1ull << lane));
    if (!one_bucket) wave_split(S, m, d0, lane, le & ~(1ull << lane));
  }
  // The first groups: runs of equal digits d and d + 1 after two splits, of
  // equal digit d in a chunk of buckets, the whole chunk when unsplit; a
  // suffix alone in its group is finished.  The kept suffixes form the live
  // list (positions ascending): gr[x] is the group of entry x, hp[g] the
  // first entry of group g (hp[groups] = n), bit j of headw marks a group
  // starting at position j.
  // (In chunks of 3 a lane the first drop is left to the loop, with a pass
  // of its own for the heads: that measures faster there.)
  const uint64_t hmask = two ? (digit_mask(d0) | digit_mask(d0 + 1)) : (ch.unsplit ? 0ull : digit_mask(d0));
  uint32_t n = 0;        // live-list length
  uint32_t ngroups = 0;  // groups of the live list
  if (!SPLIT_CHUNKS) {
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      const uint32_t j = i * LOCAL_WG + lane;
      bool h = false;
      if (j < m) {
        h = j == 0 || (!ch.unsplit && digit_of(S.K[j], d0) != digit_of(S.K[j - 1], d0));
        S.live[j] = (uint16_t)j;
      }
      const uint64_t hm = __ballot(h);
      if (lane == 0) {
        S.headw[2 * i] = (uint32_t)hm;
        S.headw[2 * i + 1] = (uint32_t)(hm >> 32);
      }
    }
    n = m;
  } else {
    uint32_t run = 0;
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      if (i * LOCAL_WG >= (int)m) break;
      const uint32_t j = i * LOCAL_WG + lane;
      bool keep = false, h = false;
      if (j < m) {
        const uint64_t kj = S.K[j];
        h = j == 0 || ((kj ^ S.K[j - 1]) & hmask) != 0;
        const bool hn = j + 1 >= m || ((S.K[j + 1] ^ kj) & hmask) != 0;
        keep = !(h && hn);
      }
      const uint64_t hm = __ballot(h);
      if (lane == 0) {
        S.headw[2 * i] = (uint32_t)hm;
        S.headw[2 * i + 1] = (uint32_t)(hm >> 32);
      }
      const uint64_t kb = __ballot(keep);
      const uint64_t hb = __ballot(keep && h);
      if (keep) {
        const uint32_t xn = n + (uint32_t)__popcll(kb & (le >> 1));
        const uint32_t g = run + (uint32_t)__popcll(hb & le) - 1u;
        S.live[xn] = (uint16_t)j;
        S.gr[xn] = (uint16_t)g;
        if (h) S.hp[g] = (uint16_t)xn;
      }
      n += (uint32_t)__popcll(kb);
      run += (uint32_t)__popcll(hb);
    }
    if (lane == 0) S.hp[run] = (uint16_t)n;
    ngroups = run;
  }
  __syncthreads();
  uint32_t r = ch.r;
  bool fetch_round = false;  // every round after the first sort fetches a window
  for (;;) {
    if (SPLIT_CHUNKS && !fetch_round) {
      if (n == 0) break;
    } else {
      // drop the finished groups: single suffixes, and (after a sort) runs
      // of equal keys that end inside the window, i.e. identical suffixes.
      // A group is a run of live entries from a head to the next head, so an
      // entry is alone in its group when it and the next live entry are both heads;
      // the other test is the same for every member of a group of equal
      // keys, so whole groups stay or go.  The groups of the kept list are
      // made in the same pass (a group is kept or dropped whole, so its head
      // is its first kept entry).  The heads of the groups the last sort
      // made are found here too: a live entry that is not a head has its
      // group's entry at the position before it, and starts a new group
      // where the two keys differ; an entry that is not a head and follows
      // entry x in the list is at the position after it.  A new head is
      // written for the later rounds; every lane that reads that flag in
      // this pass finds the same result from the keys.
      uint32_t kept = 0, run = 0;
#pragma unroll
      for (int i = 0; i < LI; ++i) {
        if (i * LOCAL_WG >= (int)n) break;
        const uint32_t x = i * LOCAL_WG + lane;
        bool keep = false, hd = false, fresh = false;
        uint16_t pos = 0;
        if (x < n) {
          pos = S.live[x];
          const uint64_t kp = S.K[pos];
          hd = head_at(S, pos);
          if (fetch_round && !hd) fresh = hd = order_bits(kp) != order_bits(S.K[pos - 1]);
          // entry x + 1 is read before any slot writes an index above x
          bool next_hd = true;
          if (x + 1 < n) {
            const uint32_t p1 = S.live[x + 1];
            next_hd = head_at(S, p1);
            if (fetch_round && !next_hd) next_hd = order_bits(S.K[p1]) != order_bits(kp);
          }
          keep = !(hd && next_hd) && (!fetch_round || clamp_of(kp) == (uint32_t)W);
        }
        const uint64_t kb = __ballot(keep);
        const uint64_t hb = __ballot(keep && hd);
        // compaction moves entries down only, so slot i never overwrites an
        // entry a later slot still has to read
        if (keep) {
          const uint32_t xn = kept + (uint32_t)__popcll(kb & (le >> 1));
          const uint32_t g = run + (uint32_t)__popcll(hb & le) - 1u;
          S.live[xn] = pos;
          S.gr[xn] = (uint16_t)g;
          if (hd) S.hp[g] = (uint16_t)xn;
          if (fresh) atomicOr(&S.headw[pos >> 5], 1u << (pos & 31u));
        }
        kept += (uint32_t)__popcll(kb);
        run += (uint32_t)__popcll(hb);
      }
      n = kept;
      ngroups = run;
      if (n == 0) break;
      if (lane == 0) S.hp[run] = (uint16_t)n;
      __syncthreads();
    }
    if (fetch_round) {
      if (r + 1 > rmax) {
        if (lane == 0) atomicOr(status, ST_WINDOW_BOUND);
        break;
      }
      ++r;
      // fetch the next window of every live suffix, FETCH_BATCH loads in
      // flight per lane: the positions of a batch first (a table load in a
      // build with wide positions), then every record load, then their use
      // (an entry past the list loads record 0 and is not used)
      for (uint32_t x0 = 0; x0 < n; x0 += FETCH_BATCH * LOCAL_WG) {
        TextRec tr[FETCH_BATCH];
        uint32_t tp[FETCH_BATCH];
        uint64_t pp[FETCH_BATCH];
#pragma unroll
        for (int i = 0; i < FETCH_BATCH; ++i) {
          const uint32_t x = x0 + i * LOCAL_WG + lane;
          tp[i] = S.live[x < n ? x : 0];
          pp[i] = S.H[tp[i]];
        }
        if (pos64) {
#pragma unroll
          for (int i = 0; i < FETCH_BATCH; ++i) pp[i] = pos64[pp[i]];
        }
#pragma unroll
        for (int i = 0; i < FETCH_BATCH; ++i) {
          const uint32_t x = x0 + i * LOCAL_WG + lane;
          tr[i] = window_load(text, nb, x < n ? pp[i] : 0, x < n ? r : 0);
        }
#pragma unroll
        for (int i = 0; i < FETCH_BATCH; ++i) {
          const uint32_t x = x0 + i * LOCAL_WG + lane;
          if (x < n) {
            const uint32_t j = tp[i];
            S.K[j] = window_combine(tr[i], nb, pp[i], r, (uint32_t)S.K[j] & 7u);
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
    // In the first sort after two splits from digit d >= 2 every group
    // agrees in digits 0..3, the high words of its keys: the low words decide
    // (oj + 8 does not carry out of them, its bits 9..8 being zero).
    bool big_groups = false;
    const bool low_words = !fetch_round && two && d0 >= 2;
    for (uint32_t x = lane; x < n; x += LOCAL_WG) {
      const uint32_t j = S.live[x];
      const uint32_t g = S.gr[x];
      const uint32_t x0 = S.hp[g];
      const uint32_t a = S.live[x0];
      const uint32_t e = a + ((uint32_t)S.hp[g + 1] - x0);  // a group is a run of positions
      if (SORT_BIG && e - a > BIG_GROUP) {
        // sorted in place below: stays where it is for now
        S.gr[x] = (uint16_t)j;
        big_groups = true;
        continue;
      }
      const uint64_t oj = order_bits(S.K[j]);
      const uint64_t below = oj + 8;  // cannot wrap: key bits 9..8 are zero
      // four independent LDS reads per step keep the loops off the
      // load-latency chain
      uint32_t c = 0;
      if (low_words) {
        c = count_below<uint32_t, 2>((const uint32_t *)S.K, a, j, e, (uint32_t)below, (uint32_t)oj);
      } else if (LI > 3) {
        c = count_below<uint64_t, 1>(S.K, a, j, e, below, oj);
      } else {
        // (small chunks, small groups: index loops measure faster here)
        uint32_t t = a;
        for (; t + 4 <= j; t += 4)
          c += (uint32_t)(S.K[t] < below) + (uint32_t)(S.K[t + 1] < below) + (uint32_t)(S.K[t + 2] < below) +
               (uint32_t)(S.K[t + 3] < below);
        for (; t < j; ++t) c += (uint32_t)(S.K[t] < below);
        for (; t + 4 <= e; t += 4)
          c += (uint32_t)(S.K[t] < oj) + (uint32_t)(S.K[t + 1] < oj) + (uint32_t)(S.K[t + 2] < oj) +
               (uint32_t)(S.K[t + 3] < oj);
        for (; t < e; ++t) c += (uint32_t)(S.K[t] < oj);
      }
      S.gr[x] = (uint16_t)(a + c);
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
          sd[i] = S.gr[x];
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
    if (SORT_BIG && __ballot(big_groups)) sort_big_groups(S, ngroups, lane);
    // (the new group heads, changes of the full key, are found by the next
    // pass over the list)
    fetch_round = true;
  }
  // a4: emit, as emit_row does, in phases: the BWT bytes; the positions of
  // the offset-0 suffixes (preceded by '$'); every load of their read ranks;
  // the rows.  Entries that are not offset-0 suffixes load position 0 and
  // write nothing.
  {
    const uint32_t lut = 'A' | ('C' << 8) | ('G' << 16) | ('T' << 24);
    uint64_t ep[LI];
    bool first[LI];
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      const uint32_t j = i * LOCAL_WG + lane;
      first[i] = false;
      ep[i] = 0;
      if (j < m) {
        const uint32_t pv = (uint32_t)S.K[j] & 7u;
        bwt[ch.start + j + cm.out_shift] = pv == 4 ? (uint8_t)'$' : (uint8_t)((lut >> (8 * pv)) & 0xFFu);
        first[i] = pv == 4;
        if (first[i]) ep[i] = S.H[j];
      }
    }
    if (pos64) {
#pragma unroll
      for (int i = 0; i < LI; ++i) ep[i] = first[i] ? pos64[ep[i]] : 0;
    }
    uint64_t lo[LI];
    uint32_t sr[LI];
#pragma unroll
    for (int i = 0; i < LI; ++i) {
      lo[i] = text[ep[i] >> 4].lo;
      sr[i] = srank[ep[i] >> 4];
    }
#pragma unroll
    for (int i = 0; i < LI; ++i)
      if (first[i]) {
        const uint32_t rank = sr[i] + (uint32_t)__popcll(lo[i] & ((1ull << (ep[i] & 15)) - 1ull));
        start_row[rank] = (uint64_t)((int64_t)(ch.start + i * LOCAL_WG + lane) + cm.row_shift);
      }
  }
  if (!PERSIST) break;
  }
  nfetch = wave_incl_sum(nfetch);
  if (lane == 63 && nfetch) atomicAdd(stat_slot(fetches), (unsigned long long)nfetch);
}


// ---------------------------------------------------------------------------
// f1: the build in ranges of window-0 key prefixes (Section 3.1's ell-prefix
// partitions, Fig. 2 steps 1-3).  A counting pass gives the sizes of the
// prefix classes, oversize classes are refined one digit deeper, and runs of
// consecutive classes form ranges of at most a budget of suffixes.  Each
// range is listed from the text on its own (a scan of every position), sorted
// by the levels and chunks like a whole collection, and emitted at the rows
// after the ranges before it: concatenating the ranges in key order gives
// the BWT, so the sort buffers need only hold one range.
// ---------------------------------------------------------------------------
constexpr int PH_MAX_PREFIXES = 48;  // prefixes refined by one counting pass (48 KB of LDS counters)
constexpr int LIST_ITEMS = 16;       // positions per thread of a listing tile (one text record)
constexpr int LIST_TILE = BLOCK * LIST_ITEMS;

// Top `depth` digits of the ordering bits of a window-0 key (depth 0..8;
// digit 7 is the clamped length, so depth 8 keeps every ordering bit).
__device__ __forceinline__ uint64_t prefix_of(uint64_t k, uint32_t depth) {
  return depth == 0 ? 0ull : depth >= 8 ? (k & ~7ull) : (k & (~0ull << (64 - 8 * depth)));
}

// Counts of digit `depth` of the window-0 keys of the suffixes whose keys
// begin with one of the np prefixes of `depth` digits (ascending; depth 0:
// one empty prefix, every suffix): counts[i * 256 + digit] for prefix i.
// Per-workgroup LDS counters (np * 256), added to the totals once.
__global__ __launch_bounds__(BLOCK) void k_prefix_hist(const TextRec *__restrict__ text, uint64_t nb,
                                                       const uint64_t *__restrict__ prefixes, uint32_t np,
                                                       uint32_t depth, unsigned long long *__restrict__ counts) {
  extern __shared__ uint32_t ph_lds[];
  uint32_t *h = ph_lds;
  uint64_t *pf = (uint64_t *)(ph_lds + np * 256);
  for (uint32_t i = threadIdx.x; i < np * 256; i += BLOCK) h[i] = 0;
  if (threadIdx.x < np) pf[threadIdx.x] = prefixes[threadIdx.x];
  __syncthreads();
  const uint64_t nrec = (nb + 15) / 16;
  for (uint64_t w = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; w < nrec; w += (uint64_t)gridDim.x * BLOCK) {
    const TextRec t = text[w];
    const uint64_t p0 = 16 * w;
    for (uint32_t o = 0; o < 16 && p0 + o < nb; ++o) {
      const uint64_t p = p0 + o;
      uint32_t prev3 = 4;
      if (!((t.lo >> o) & 1u)) prev3 = o ? rec_base_at(t, o - 1) : (uint32_t)(t.lo >> 42) & 3u;
      const uint64_t k = window_combine(t, nb, p, 0, prev3);
      const uint64_t top = prefix_of(k, depth);
      uint32_t lo = 0, hi = np;  // first prefix >= top
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pf[mid] < top) lo = mid + 1;
        else hi = mid;
      }
      if (lo < np && pf[lo] == top) atomicAdd(&h[lo * 256 + digit_of(k, (int)depth)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < np * 256; i += BLOCK)
    if (h[i]) atomicAdd(&counts[i], (unsigned long long)h[i]);
}

// Window-0 keys of the 16 positions of record w into k[], with a bit per
// position in range [lo, hi] (ordering bits) in the result.
__device__ __forceinline__ uint32_t record_keys_in_range(const TextRec *__restrict__ text, uint64_t nb, uint64_t w,
                                                         uint64_t lo, uint64_t hi, uint64_t (&k)[LIST_ITEMS]) {
  uint32_t in = 0;
  const uint64_t p0 = 16 * w;
  if (p0 >= nb) return 0;
  const TextRec t = text[w];
#pragma unroll
  for (uint32_t o = 0; o < LIST_ITEMS; ++o) {
    const uint64_t p = p0 + o;
    uint32_t prev3 = 4;
    if (!((t.lo >> o) & 1u)) prev3 = o ? rec_base_at(t, o - 1) : (uint32_t)(t.lo >> 42) & 3u;
    k[o] = window_combine(t, nb, p, 0, prev3);
    const uint64_t ob = order_bits(k[o]);
    if (p < nb && ob >= lo && ob <= hi) in |= 1u << o;
  }
  return in;
}

// Suffixes of a range per listing tile (LIST_TILE positions, thread t owning
// record tile * BLOCK + t).
__global__ __launch_bounds__(BLOCK) void k_range_count(const TextRec *__restrict__ text, uint64_t nb, uint64_t lo,
                                                       uint64_t hi, uint32_t *__restrict__ tile_count) {
  __shared__ uint32_t tmp[WAVES];
  uint64_t k[LIST_ITEMS];
  const uint64_t w = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t c = (uint32_t)__popc(record_keys_in_range(text, nb, w, lo, hi, k));
  uint32_t total;
  block_excl_sum(c, tmp, &total);
  if (threadIdx.x == 0) tile_count[blockIdx.x] = total;
}

// In place: exclusive prefix sums of n counts, per block of BLOCK *
// RANK_WPT counts, and each block's total in blocksum (k_rank_top then
// scans the block totals).
__global__ __launch_bounds__(BLOCK) void k_count_blocks(const uint32_t *__restrict__ cnt, uint64_t n,
                                                        uint32_t *__restrict__ blocksum) {
  __shared__ uint32_t tmp[WAVES];
  const uint64_t i0 = (uint64_t)blockIdx.x * RANK_BLOCK_WORDS + (uint64_t)threadIdx.x * RANK_WPT;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < RANK_WPT; ++i)
    if (i0 + i < n) c += cnt[i0 + i];
  uint32_t total;
  block_excl_sum(c, tmp, &total);
  if (threadIdx.x == 0) blocksum[blockIdx.x] = total;
}
__global__ __launch_bounds__(BLOCK) void k_count_prefix(uint32_t *__restrict__ cnt, uint64_t n,
                                                        const uint32_t *__restrict__ blocksum) {
  __shared__ uint32_t tmp[WAVES];
  const uint64_t i0 = (uint64_t)blockIdx.x * RANK_BLOCK_WORDS + (uint64_t)threadIdx.x * RANK_WPT;
  uint32_t v[RANK_WPT];
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < RANK_WPT; ++i) {
    v[i] = i0 + i < n ? cnt[i0 + i] : 0u;
    c += v[i];
  }
  uint32_t run = blocksum[blockIdx.x] + block_excl_sum(c, tmp, nullptr);
#pragma unroll
  for (int i = 0; i < RANK_WPT; ++i) {
    if (i0 + i < n) cnt[i0 + i] = run;
    run += v[i];
  }
}

// The range's suffixes in position order (read order, so equal suffixes
// keep the read-index order the stable passes preserve): window-0 key and
// handle at tile_start[tile] + rank in the tile - skip, for the members of
// rank skip .. skip + take - 1 (a piece of a class of identical suffixes;
// skip 0 and take = all for a whole range).
__global__ __launch_bounds__(BLOCK) void k_range_list(const TextRec *__restrict__ text, uint64_t nb, uint64_t lo,
                                                      uint64_t hi, const uint32_t *__restrict__ tile_start,
                                                      uint64_t skip, uint64_t take, uint64_t *__restrict__ keys,
                                                      uint32_t *__restrict__ hdl, uint64_t *__restrict__ pos64) {
  __shared__ uint32_t tmp[WAVES];
  uint64_t k[LIST_ITEMS];
  const uint64_t w = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t in = record_keys_in_range(text, nb, w, lo, hi, k);
  uint64_t at = (uint64_t)tile_start[blockIdx.x] + block_excl_sum((uint32_t)__popc(in), tmp, nullptr);
#pragma unroll
  for (uint32_t o = 0; o < LIST_ITEMS; ++o)
    if ((in >> o) & 1u) {
      if (at >= skip && at - skip < take) {
        const uint64_t j = at - skip;
        keys[j] = k[o];
        if (pos64) {
          pos64[j] = 16 * w + o;
          hdl[j] = (uint32_t)j;
        } else {
          hdl[j] = (uint32_t)(16 * w + o);
        }
      }
      ++at;
    }
}

// ---------------------------------------------------------------------------
// f2: the stringword schedule of Section 3.2, literally: a least-significant-
// digit radix sort of (key, handle) over every window of every suffix, the
// last window first.  Before the passes of window w each suffix's window-w
// key is computed in position order and permuted into the current order by
// its handle (the paper's permutation of the next stringword by index);
// stable passes over its eight digits, least significant first, then order
// the suffixes by (window w, windows after w).  A suffix that ended before
// window w has key 0 there, below every key of a suffix that goes on, and
// suffixes equal in every window are identical and stay in read order.
// ---------------------------------------------------------------------------

// Window-w key of the suffix at base p for the stringword schedule: the
// window's key when the suffix reaches the window's start (no read starts
// strictly inside p+1 .. q-1, q = p + 27 w), else 0; window 0 carries the
// preceding symbol.
__device__ __forceinline__ uint64_t schedule_key(const TextRec *__restrict__ text, const uint32_t *__restrict__ srank,
                                                 uint64_t nb, uint64_t p, uint32_t w) {
  if (w == 0) return first_key(text, nb, p);
  const uint64_t q = p + (uint64_t)W * w;
  if (q > nb) return 0;
  if (start_rank(text, srank, q) != start_rank(text, srank, p + 1)) return 0;
  return window_key(text, nb, p, w, 0);
}

// keyw[p] for every position (coalesced), and the OR and AND of the
// ordering bits (which digits vary).
__global__ __launch_bounds__(BLOCK) void k_sched_window(const TextRec *__restrict__ text,
                                                        const uint32_t *__restrict__ srank, uint64_t nb, uint32_t w,
                                                        uint64_t *__restrict__ keyw, unsigned long long *orand) {
  __shared__ uint64_t red[WAVES];
  uint64_t o = 0, a = ~0ull;
  for (uint64_t p = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; p < nb; p += (uint64_t)gridDim.x * BLOCK) {
    const uint64_t k = schedule_key(text, srank, nb, p, w);
    keyw[p] = k;
    o |= k;
    a &= k;
  }
  o = block_or(o, red);
  a = block_and(a, red);
  if (threadIdx.x == 0) {
    atomicOr(&orand[0], (unsigned long long)order_bits(o));
    atomicAnd(&orand[1], (unsigned long long)(a | 7ull));
  }
}

// K[j] = keyw[H[j]]: the window's keys in the current order (the first
// window's handles are the positions in order: H[j] = j).
__global__ __launch_bounds__(BLOCK) void k_sched_gather(const uint64_t *__restrict__ keyw, uint64_t nb, bool first,
                                                        uint64_t *__restrict__ K, uint32_t *__restrict__ H) {
  const uint64_t stride = (uint64_t)gridDim.x * BLOCK;
  if (first) {
    for (uint64_t j = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; j < nb; j += stride) {
      H[j] = (uint32_t)j;
      K[j] = keyw[j];
    }
    return;
  }
  // four gathers in flight per thread: the handles, then the keys they name
  constexpr int G = 4;
  for (uint64_t j0 = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; j0 < nb; j0 += G * stride) {
    uint32_t h[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint64_t j = j0 + g * stride;
      h[g] = H[j < nb ? j : nb - 1];
    }
    uint64_t k[G];
#pragma unroll
    for (int g = 0; g < G; ++g) k[g] = keyw[h[g]];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint64_t j = j0 + g * stride;
      if (j < nb) K[j] = k[g];
    }
  }
}

// Per-tile counts of digit d (tile of TL suffixes).
template <int TL>
__global__ __launch_bounds__(BLOCK) void k_sched_hist(const uint64_t *__restrict__ K, uint64_t nb, int d,
                                                      uint32_t *__restrict__ tile_hist) {
  __shared__ uint32_t hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t t0 = (uint64_t)blockIdx.x * TL;
  constexpr int PER = TL / BLOCK;
  // every key load of the tile first (an item past the end reads the last
  // key, nb > t0), then the counts
  uint64_t kk[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint64_t j = t0 + (uint64_t)i * BLOCK + threadIdx.x;
    kk[i] = K[j < nb ? j : nb - 1];
  }
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (t0 + (uint64_t)i * BLOCK + threadIdx.x < nb) atomicAdd(&hist[digit_of(kk[i], d)], 1u);
  __syncthreads();
  tile_hist[(uint64_t)blockIdx.x * 256 + threadIdx.x] = hist[threadIdx.x];
}

// After k_group_scan over one segment of all tiles: the group totals become
// each (group, digit) run's first output position, digit-major (all of
// digit 0 first).  One wave; lane l holds digits l, 64 + l, 128 + l, 192 + l.
__global__ __launch_bounds__(64) void k_sched_top(uint32_t *__restrict__ gsum, uint32_t ngroups) {
  uint32_t cv[4] = {0u, 0u, 0u, 0u};
  group_totals(gsum, 0, ngroups, cv);
  uint32_t run[4];
  uint32_t carry = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t incl = wave_incl_sum(cv[i]);
    run[i] = carry + incl - cv[i];
    carry += (uint32_t)__shfl((int)incl, 63, 64);
  }
  group_starts(gsum, 0, ngroups, run);
}

// One stable pass by digit d: tile t of Ki/Hi to Ko/Ho.
template <int TI, int NW>
__global__ __launch_bounds__(64 * NW) void k_sched_scatter(const uint64_t *__restrict__ Ki,
                                                           const uint32_t *__restrict__ Hi, uint64_t nb, int d,
                                                           const uint32_t *__restrict__ tile_hist,
                                                           const uint32_t *__restrict__ gsum, uint64_t *__restrict__ Ko,
                                                           uint32_t *__restrict__ Ho) {
  constexpr uint32_t TL = 64 * NW * TI;
  __shared__ ScatterSmem<TI, NW> S;
  const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const uint64_t t0 = (uint64_t)tile * TL;
  const uint32_t m = (uint32_t)min((uint64_t)TL, nb - t0);
  uint64_t kr[TI];
  uint32_t hr[TI], dig[TI];
  // every load of the tile is issued before any is used (an item past the
  // tile reads the last one, m >= 1, and is then cleared)
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const uint32_t li = item_index<TI>(i);
    const uint64_t at = t0 + (li < m ? li : m - 1);
    kr[i] = Ki[at];
    hr[i] = Hi[at];
  }
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    if (item_index<TI>(i) < m) {
      dig[i] = digit_of(kr[i], d);
    } else {
      kr[i] = 0;
      hr[i] = 0;
      dig[i] = NODIGIT;
    }
  }
  const uint32_t g = tile / GROUP_TILES;
  if (threadIdx.x < 256)
    S.goff[threadIdx.x] = (uint64_t)gsum[(uint64_t)g * 256 + threadIdx.x] + tile_hist[(uint64_t)tile * 256 + threadIdx.x];
  tile_scatter(S, kr, hr, dig, m, d, Ko, Ho);
}

// The sorted suffixes' BWT rows (window-0 keys carry the preceding symbol).
__global__ __launch_bounds__(BLOCK) void k_sched_emit(const uint64_t *__restrict__ K, const uint32_t *__restrict__ H,
                                                      uint64_t nb, const CollMap *__restrict__ cmap,
                                                      const TextRec *__restrict__ text,
                                                      const uint32_t *__restrict__ srank, uint8_t *__restrict__ bwt,
                                                      uint64_t *__restrict__ start_row) {
  const CollMap cm = cmap[0];
  for (uint64_t j = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; j < nb; j += (uint64_t)gridDim.x * BLOCK)
    emit_row(j, cm, K[j], H[j], nullptr, text, srank, bwt, start_row);
}

}  // namespace
