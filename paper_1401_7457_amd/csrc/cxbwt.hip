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
//   * key     = one 28-base window of the suffix: 56 bits of bases (zero past
//               the end of the read), 5 bits holding min(remaining, 28), and
//               3 bits carrying the symbol that precedes the suffix (0..3 a
//               base, 4 = '$').  Ordering uses bits [3, 64) only.  Comparing
//               (bases, clamped length) lexicographically is the order of
//               Section 2 within one window: a suffix that ends inside the
//               window is a proper prefix of, hence below, one that goes on;
//               equal keys with a clamped length below 28 are identical
//               suffixes, which stable passes keep in read order.
//   * sort    = most-significant-digit first: global 8-bit digit levels split
//               the key space until every bucket fits one workgroup (4096
//               suffixes); each bucket set is then sorted, refined and emitted
//               entirely in LDS.  A tie on a full window (clamped length 28)
//               fetches the next window of the tied suffixes only.
//
// Every pass is stable and the initial order is read-major, so suffixes that
// are equal through their terminators stay in read-index order (Section 3.2's
// stability argument).

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "cxbwt.h"

namespace {

// ---------------------------------------------------------------------------
// constants
// ---------------------------------------------------------------------------
constexpr int W = 28;                    // bases per key window
constexpr int BLOCK = 256;               // threads per workgroup
constexpr int WAVES = BLOCK / 64;        // wave64
constexpr int ITEMS = 16;                // suffixes per thread in a tile
constexpr int TILE = BLOCK * ITEMS;      // 4096: tile of a global level
constexpr int WAVE_SPAN = 64 * ITEMS;    // suffixes per wave in a tile
constexpr int CHUNK = 4096;              // largest bucket set finished in LDS
constexpr int RANK_COUNT_MAX = 256;      // live groups up to this size: all-pairs ranking
constexpr uint32_t NODIGIT = 0xFFFFFFFFu;

constexpr uint32_t ST_BAD_OFFSETS = 1u;
constexpr uint32_t ST_TOO_LONG = 2u;
constexpr uint32_t ST_BAD_CHAR = 4u;
constexpr uint32_t ST_LIST_OVERFLOW = 8u;
constexpr uint32_t ST_WINDOW_BOUND = 16u;

static_assert(TILE == CHUNK, "tile and chunk share the register layout");

// A run of suffixes [start, start+len) in key/handle buffer `buf`, whose keys
// are for window r and agree on every digit before d.
struct Seg {
  uint64_t start;
  uint64_t len;
  uint32_t r;
  uint8_t d;
  uint8_t buf;
  uint8_t regather;  // keys must be re-fetched for window r before use
  uint8_t pad;
};

struct Lists {
  Seg *big_next;
  uint32_t *n_big_next;
  uint32_t cap_big;
  Seg *chunks;
  uint32_t *n_chunks;
  uint32_t cap_chunks;
  Seg *finals;
  uint32_t *n_finals;
  uint32_t cap_finals;
  uint32_t *status;
  uint32_t rmax;
};

// ---------------------------------------------------------------------------
// key helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t order_bits(uint64_t k) { return k & ~7ull; }
__device__ __forceinline__ uint32_t clamp_of(uint64_t k) { return (uint32_t)(k >> 3) & 31u; }
__device__ __forceinline__ uint32_t digit_of(uint64_t k, int j) {
  return j < 7 ? (uint32_t)(k >> (56 - 8 * j)) & 0xFFu : (uint32_t)(k >> 3) & 0x1Fu;
}
__host__ __device__ __forceinline__ uint64_t digit_mask(int j) {
  return j < 7 ? (0xFFull << (56 - 8 * j)) : (0x1Full << 3);
}
__device__ __forceinline__ uint32_t base_at(const uint64_t *packed, uint64_t t) {
  return (uint32_t)(packed[t >> 5] >> (62 - 2 * (t & 31))) & 3u;
}
__device__ __forceinline__ bool end_bit(const uint64_t *endbits, uint64_t t) {
  return (endbits[t >> 6] >> (t & 63)) & 1ull;
}

// Key of window r of the suffix whose first base is p (the window starts at
// base q = p + 28 r).  endbits marks the last base of every non-empty read.
// For r >= 1 the caller guarantees the read still holds at least 28 r bases
// from p, so the read's last base e satisfies e >= q - 1.
__device__ uint64_t window_key(const uint64_t *__restrict__ packed, const uint64_t *__restrict__ endbits,
                               uint64_t nb, uint64_t p, uint32_t r, uint32_t prev3) {
  uint64_t q = p + (uint64_t)W * r;
  uint64_t lo = r == 0 ? p : q - 1;
  if (lo >= nb) return prev3;  // never taken for a live suffix; keeps reads in bounds
  uint64_t w0 = endbits[lo >> 6] >> (lo & 63);
  uint64_t e;
  if (w0) {
    e = lo + (uint64_t)__builtin_ctzll(w0);
  } else {
    uint64_t b1 = (lo | 63ull) + 1;
    uint64_t w1 = endbits[b1 >> 6];
    e = w1 ? b1 + (uint64_t)__builtin_ctzll(w1) : ~0ull;
  }
  uint32_t clamp = (e < q + W) ? (uint32_t)(e + 1 - q) : (uint32_t)W;
  uint64_t chars = 0;
  if (clamp > 0 && q < nb) {
    uint64_t wi = q >> 5;
    uint32_t b = 2u * (uint32_t)(q & 31);
    uint64_t x = packed[wi] << b;
    if (b) x |= packed[wi + 1] >> (64 - b);
    chars = x & ~0xFFull;
    if (clamp < (uint32_t)W) chars &= ~((1ull << (64 - 2 * clamp)) - 1);
  }
  return chars | ((uint64_t)clamp << 3) | prev3;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (l >= (uint32_t)o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint64_t wave_and(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v &= __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
  return v;
}

// Exclusive prefix sum of one value per thread over the workgroup.
__device__ uint32_t block_excl_sum(uint32_t v, uint32_t *tmp, uint32_t *total) {
  uint32_t inc = wave_incl_sum(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) tmp[w] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) {
    uint32_t x = tmp[i];
    if (i < w) pre += x;
    tot += x;
  }
  __syncthreads();
  if (total) *total = tot;
  return pre + inc - v;
}

__device__ uint64_t block_or(uint64_t v, uint64_t *tmp) {
  v = wave_or(v);
  if (lane_id() == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) r |= tmp[i];
  __syncthreads();
  return r;
}
__device__ uint64_t block_and(uint64_t v, uint64_t *tmp) {
  v = wave_and(v);
  if (lane_id() == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = ~0ull;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) r &= tmp[i];
  __syncthreads();
  return r;
}
__device__ uint32_t block_max(uint32_t v, uint32_t *tmp) {
  v = wave_max(v);
  if (lane_id() == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) r = max(r, tmp[i]);
  __syncthreads();
  return r;
}

// Index of the ITEMS items of this thread in a tile: wave w owns
// [w*WAVE_SPAN, (w+1)*WAVE_SPAN); item i of lane l is w*WAVE_SPAN + i*64 + l.
__device__ __forceinline__ uint32_t item_index(int i) {
  return (uint32_t)((threadIdx.x >> 6) * WAVE_SPAN + i * 64) + lane_id();
}

// Stable 256-way split of up to TILE items held in registers (layout of
// item_index).  On return pos[i] is the destination of item i in [0, count);
// dstart[d] is the first destination of digit d.  dig[i] == NODIGIT marks an
// absent item.
__device__ void block_multisplit(const uint32_t (&dig)[ITEMS], uint32_t (&pos)[ITEMS], uint32_t *wcount,
                                 uint32_t *dstart, uint32_t *tmp) {
  const int w = threadIdx.x >> 6;
  for (int x = threadIdx.x; x < WAVES * 256; x += BLOCK) wcount[x] = 0;
  __syncthreads();
  uint32_t *wc = wcount + w * 256;
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t d = dig[i];
    const bool valid = d != NODIGIT;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t v = __ballot(bit);
      peers &= bit ? v : ~v;
    }
    if (valid) {
      const uint32_t before = wc[d];
      pos[i] = before + (uint32_t)__popcll(peers & lt);
      if ((peers & lt) == 0) wc[d] = before + (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();
  const uint32_t d = threadIdx.x;  // BLOCK == 256 digits
  uint32_t run = 0;
#pragma unroll
  for (int ww = 0; ww < WAVES; ++ww) {
    const uint32_t c = wcount[ww * 256 + d];
    wcount[ww * 256 + d] = run;
    run += c;
  }
  const uint32_t ex = block_excl_sum(run, tmp, nullptr);
  dstart[d] = ex;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (dig[i] != NODIGIT) pos[i] += dstart[dig[i]] + wc[dig[i]];
}

// Writes the BWT row of a sorted suffix and, for an offset-0 suffix, the
// row into term_pos of its read (the read whose first base is p).
__device__ __forceinline__ void emit_row(uint64_t row, uint64_t key, uint32_t p, const uint64_t *__restrict__ offsets,
                                         uint64_t n, uint8_t *__restrict__ bwt, uint64_t *__restrict__ term_pos) {
  const uint32_t pv = (uint32_t)key & 7u;
  const uint32_t lut = 'A' | ('C' << 8) | ('G' << 16) | ('T' << 24);
  bwt[row] = pv == 4 ? (uint8_t)'$' : (uint8_t)((lut >> (8 * pv)) & 0xFFu);
  if (pv == 4) {
    // largest i with offsets[i] <= p: the read that starts at p
    uint64_t lo = 0, hi = n;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (offsets[mid] <= (uint64_t)p) lo = mid;
      else hi = mid;
    }
    term_pos[lo] = row;
  }
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
__global__ void k_pack(const uint8_t *__restrict__ ascii, uint64_t nb, uint64_t *__restrict__ packed, uint64_t nwords,
                       uint32_t *status) {
  const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwords) return;
  const uint64_t t0 = w * 32;
  uint64_t x = 0;
  bool bad = false;
  for (int j = 0; j < 32; ++j) {
    const uint64_t t = t0 + j;
    if (t >= nb) break;
    const uint8_t c = ascii[t];
    uint64_t code;
    switch (c) {
      case 'A': code = 0; break;
      case 'C': code = 1; break;
      case 'G': code = 2; break;
      case 'T': code = 3; break;
      default: code = 0; bad = true; break;
    }
    x |= code << (62 - 2 * j);
  }
  packed[w] = x;
  if (bad && status) atomicOr(status, ST_BAD_CHAR);
}

// ---------------------------------------------------------------------------
// read preparation: validate offsets, mark read ends, emit the n rows of the
// bare terminators (row i = $_i, preceded by the last base of read i)
// ---------------------------------------------------------------------------
__global__ void k_prep(const uint64_t *__restrict__ packed, const uint64_t *__restrict__ offsets, uint64_t n, uint64_t nb,
                       uint32_t maxlen, unsigned long long *endbits, uint8_t *__restrict__ bwt,
                       uint64_t *__restrict__ term_pos, uint32_t *status) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t a = offsets[i], b = offsets[i + 1];
  bool bad = b < a || b > nb || (i == 0 && a != 0) || (i == n - 1 && b != nb);
  if (bad) {
    atomicOr(status, ST_BAD_OFFSETS);
    return;
  }
  if (b - a > (uint64_t)maxlen) {
    atomicOr(status, ST_TOO_LONG);
    return;
  }
  if (b > a) {
    const uint64_t e = b - 1;
    atomicOr(&endbits[e >> 6], 1ull << (e & 63));
    const uint32_t lut = 'A' | ('C' << 8) | ('G' << 16) | ('T' << 24);
    bwt[i] = (uint8_t)((lut >> (8 * base_at(packed, e))) & 0xFFu);
  } else {
    bwt[i] = (uint8_t)'$';
    term_pos[i] = i;
  }
}

// ---------------------------------------------------------------------------
// a1: suffix listing + window-0 keys, read-major (handle = base position)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_gen(const uint64_t *__restrict__ packed, const uint64_t *__restrict__ endbits,
                                               uint64_t nb, uint64_t *__restrict__ keys, uint32_t *__restrict__ hdl) {
  const uint64_t p = (uint64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (p >= nb) return;
  uint32_t prev3;
  if (p == 0 || end_bit(endbits, p - 1)) prev3 = 4;
  else prev3 = base_at(packed, p - 1);
  keys[p] = window_key(packed, endbits, nb, p, 0, prev3);
  hdl[p] = (uint32_t)p;
}

// ---------------------------------------------------------------------------
// a2/a3 global levels: split every oversized segment by one 8-bit digit
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t find_seg(const uint32_t *tile_prefix, uint32_t nsegs, uint32_t tile) {
  uint32_t lo = 0, hi = nsegs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tile_prefix[mid] <= tile) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Per-tile digit histogram and per-segment OR/AND of the ordering bits.  A
// segment flagged `regather` first re-fetches its keys for window r.
__global__ __launch_bounds__(BLOCK) void k_level_hist(const Seg *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                                                      uint32_t nsegs, uint64_t *keys0, uint64_t *keys1,
                                                      const uint32_t *__restrict__ hdl0, const uint32_t *__restrict__ hdl1,
                                                      const uint64_t *__restrict__ packed,
                                                      const uint64_t *__restrict__ endbits, uint64_t nb,
                                                      uint32_t *__restrict__ tile_hist, unsigned long long *seg_or,
                                                      unsigned long long *seg_and) {
  __shared__ uint32_t hist[256];
  const uint32_t tile = blockIdx.x;
  const uint32_t s = find_seg(tile_prefix, nsegs, tile);
  const Seg sg = segs[s];
  const uint64_t t0 = sg.start + (uint64_t)(tile - tile_prefix[s]) * TILE;
  const uint64_t t1 = min(t0 + (uint64_t)TILE, sg.start + sg.len);
  uint64_t *K = sg.buf ? keys1 : keys0;
  const uint32_t *H = sg.buf ? hdl1 : hdl0;
  hist[threadIdx.x] = 0;
  __syncthreads();
  uint64_t o = 0, a = ~0ull;
  for (uint64_t j = t0 + threadIdx.x; j < t1; j += BLOCK) {
    uint64_t k = K[j];
    if (sg.regather) {
      k = window_key(packed, endbits, nb, H[j], sg.r, (uint32_t)k & 7u);
      K[j] = k;
    }
    atomicAdd(&hist[digit_of(k, sg.d)], 1u);
    o |= k;
    a &= k;
  }
  o = wave_or(o);
  a = wave_and(a);
  if (lane_id() == 0) {
    atomicOr(&seg_or[s], (unsigned long long)order_bits(o));
    atomicAnd(&seg_and[s], (unsigned long long)(a | 7ull));
  }
  __syncthreads();
  tile_hist[(uint64_t)tile * 256 + threadIdx.x] = hist[threadIdx.x];
}

__device__ void push_seg(Seg *list, uint32_t *count, uint32_t cap, const Seg &s, uint32_t *status) {
  const uint32_t at = atomicAdd(count, 1u);
  if (at < cap) list[at] = s;
  else atomicOr(status, ST_LIST_OVERFLOW);
}

// One workgroup per segment: turn tile counts into scatter offsets and sort
// the resulting buckets into: groups finished in LDS (packed into chunks of
// at most CHUNK suffixes), segments for the next level, and final groups of
// identical suffixes.  A segment whose current digit is constant is not
// scattered; it moves to its first varying digit, or, when all its ordering
// bits agree, to the next window (full tie) or to the final list (ended tie).
__global__ __launch_bounds__(BLOCK) void k_level_scan(const Seg *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                                                      uint32_t *__restrict__ tile_hist,
                                                      const unsigned long long *__restrict__ seg_or,
                                                      const unsigned long long *__restrict__ seg_and,
                                                      uint8_t *__restrict__ seg_split, Lists L) {
  __shared__ uint32_t tot[256];
  __shared__ uint32_t bstart[256];
  __shared__ uint32_t tmp[WAVES];
  __shared__ int single;
  const uint32_t s = blockIdx.x;
  const Seg sg = segs[s];
  const uint32_t tp0 = tile_prefix[s], tp1 = tile_prefix[s + 1];
  const uint32_t dg = threadIdx.x;
  uint32_t total = 0;
  for (uint32_t t = tp0; t < tp1; ++t) total += tile_hist[(uint64_t)t * 256 + dg];
  tot[dg] = total;
  if (dg == 0) single = 0;
  __syncthreads();
  if ((uint64_t)total == sg.len) single = 1;
  __syncthreads();
  if (single) {
    if (dg == 0) {
      seg_split[s] = 0;
      const uint64_t diff = (seg_or[s] ^ seg_and[s]) & ~7ull;
      Seg nx = sg;
      nx.regather = 0;
      if (diff == 0) {
        if (clamp_of(seg_and[s]) < (uint32_t)W) {
          push_seg(L.finals, L.n_finals, L.cap_finals, sg, L.status);
        } else if (sg.r + 1 > L.rmax) {
          atomicOr(L.status, ST_WINDOW_BOUND);
        } else {
          nx.r = sg.r + 1;
          nx.d = 0;
          nx.regather = 1;
          push_seg(L.big_next, L.n_big_next, L.cap_big, nx, L.status);
        }
      } else {
        const int top = 63 - __builtin_clzll(diff);
        nx.d = (uint8_t)(top >= 8 ? (63 - top) >> 3 : 7);
        push_seg(L.big_next, L.n_big_next, L.cap_big, nx, L.status);
      }
    }
    return;
  }
  const uint32_t ex = block_excl_sum(total, tmp, nullptr);
  bstart[dg] = ex;
  uint32_t run = (uint32_t)sg.start + ex;
  for (uint32_t t = tp0; t < tp1; ++t) {
    const uint64_t at = (uint64_t)t * 256 + dg;
    const uint32_t c = tile_hist[at];
    tile_hist[at] = run;
    run += c;
  }
  __syncthreads();
  if (dg == 0) {
    seg_split[s] = 1;
    Seg cur{};
    bool have = false;
    for (int b = 0; b < 256; ++b) {
      const uint32_t c = tot[b];
      if (!c) continue;
      const uint64_t st = sg.start + bstart[b];
      if (c > (uint32_t)CHUNK) {
        if (have) {
          push_seg(L.chunks, L.n_chunks, L.cap_chunks, cur, L.status);
          have = false;
        }
        Seg nx{st, c, sg.r, (uint8_t)(sg.d + 1), (uint8_t)(sg.buf ^ 1), 0, 0};
        if (sg.d == 7) {
          // bucket value b is the clamped length; all ordering bits agree
          if (b < W) {
            push_seg(L.finals, L.n_finals, L.cap_finals, nx, L.status);
          } else if (sg.r + 1 > L.rmax) {
            atomicOr(L.status, ST_WINDOW_BOUND);
          } else {
            nx.r = sg.r + 1;
            nx.d = 0;
            nx.regather = 1;
            push_seg(L.big_next, L.n_big_next, L.cap_big, nx, L.status);
          }
        } else {
          push_seg(L.big_next, L.n_big_next, L.cap_big, nx, L.status);
        }
        continue;
      }
      if (have && cur.len + c <= (uint64_t)CHUNK) {
        cur.len += c;
      } else {
        if (have) push_seg(L.chunks, L.n_chunks, L.cap_chunks, cur, L.status);
        cur = Seg{st, c, sg.r, sg.d, (uint8_t)(sg.buf ^ 1), 0, 0};
        have = true;
      }
    }
    if (have) push_seg(L.chunks, L.n_chunks, L.cap_chunks, cur, L.status);
  }
}

// Stable scatter of one tile by the segment's digit into the other buffer.
__global__ __launch_bounds__(BLOCK) void k_level_scatter(const Seg *__restrict__ segs,
                                                         const uint32_t *__restrict__ tile_prefix, uint32_t nsegs,
                                                         const uint8_t *__restrict__ seg_split,
                                                         const uint32_t *__restrict__ tile_off, uint64_t *keys0,
                                                         uint64_t *keys1, uint32_t *hdl0, uint32_t *hdl1) {
  __shared__ uint64_t sk[TILE];
  __shared__ uint32_t sh[TILE];
  __shared__ uint32_t wcount[WAVES * 256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t goff[256];
  __shared__ uint32_t tmp[WAVES];
  const uint32_t tile = blockIdx.x;
  const uint32_t s = find_seg(tile_prefix, nsegs, tile);
  if (!seg_split[s]) return;
  const Seg sg = segs[s];
  const uint64_t t0 = sg.start + (uint64_t)(tile - tile_prefix[s]) * TILE;
  const uint32_t m = (uint32_t)min((uint64_t)TILE, sg.start + sg.len - t0);
  const uint64_t *Ki = sg.buf ? keys1 : keys0;
  const uint32_t *Hi = sg.buf ? hdl1 : hdl0;
  uint64_t *Ko = sg.buf ? keys0 : keys1;
  uint32_t *Ho = sg.buf ? hdl0 : hdl1;
  const int d = sg.d;
  uint64_t kr[ITEMS];
  uint32_t hr[ITEMS], dig[ITEMS], pos[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t li = item_index(i);
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
  goff[threadIdx.x] = tile_off[(uint64_t)tile * 256 + threadIdx.x];
  block_multisplit(dig, pos, wcount, dstart, tmp);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (dig[i] != NODIGIT) {
      sk[pos[i]] = kr[i];
      sh[pos[i]] = hr[i];
    }
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < m; q += BLOCK) {
    const uint64_t k = sk[q];
    const uint32_t dd = digit_of(k, d);
    const uint64_t g = (uint64_t)goff[dd] + (q - dstart[dd]);
    Ko[g] = k;
    Ho[g] = sh[q];
  }
}

// Groups of identical suffixes too large for one workgroup: emit in place.
__global__ __launch_bounds__(BLOCK) void k_emit_final(const Seg *__restrict__ segs, const uint32_t *__restrict__ tile_prefix,
                                                      uint32_t nsegs, const uint64_t *__restrict__ keys0,
                                                      const uint64_t *__restrict__ keys1, const uint32_t *__restrict__ hdl0,
                                                      const uint32_t *__restrict__ hdl1, const uint64_t *__restrict__ offsets,
                                                      uint64_t n, uint8_t *__restrict__ bwt, uint64_t *__restrict__ term_pos) {
  const uint32_t tile = blockIdx.x;
  const uint32_t s = find_seg(tile_prefix, nsegs, tile);
  const Seg sg = segs[s];
  const uint64_t t0 = sg.start + (uint64_t)(tile - tile_prefix[s]) * TILE;
  const uint64_t t1 = min(t0 + (uint64_t)TILE, sg.start + sg.len);
  const uint64_t *K = sg.buf ? keys1 : keys0;
  const uint32_t *H = sg.buf ? hdl1 : hdl0;
  for (uint64_t j = t0 + threadIdx.x; j < t1; j += BLOCK) emit_row(n + j, K[j], H[j], offsets, n, bwt, term_pos);
}

// ---------------------------------------------------------------------------
// a2/a3/a4 in one workgroup: finish a chunk of at most CHUNK suffixes
// ---------------------------------------------------------------------------
struct LocalSmem {
  uint64_t K[2][CHUNK];
  uint32_t H[2][CHUNK];
  uint16_t G[2][CHUNK];      // group start carried through composite passes
  uint16_t gr[CHUNK];        // group rank of each position
  uint16_t hp[CHUNK + 1];    // start of each group
  uint8_t head[CHUNK];       // position starts a group
  uint8_t fin[CHUNK];        // position's group is final
  uint32_t wcount[WAVES * 256];
  uint32_t dstart[256];
  uint32_t tmp[WAVES];
  uint64_t tmp64[WAVES];
  uint32_t scan_tmp[WAVES];
};

// Stable LDS pass of m items from buffer `src` to 1-src by digit `sel`:
// 0..7 key digits (items whose group is final contribute digit 0 when
// zero_final is set, through their zeroed ordering bits), 8/9 the low/high
// byte of the carried group start.
template <bool WITH_G>
__device__ void lds_pass(LocalSmem &S, int src, uint32_t m, int sel) {
  uint64_t kr[ITEMS];
  uint32_t hr[ITEMS], dig[ITEMS], pos[ITEMS];
  uint16_t gg[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t li = item_index(i);
    if (li < m) {
      kr[i] = S.K[src][li];
      hr[i] = S.H[src][li];
      gg[i] = WITH_G ? S.G[src][li] : (uint16_t)0;
      if (sel < 8) dig[i] = digit_of(kr[i], sel);
      else if (sel == 8) dig[i] = gg[i] & 0xFFu;
      else dig[i] = (uint32_t)gg[i] >> 8;
    } else {
      kr[i] = 0;
      hr[i] = 0;
      gg[i] = 0;
      dig[i] = NODIGIT;
    }
  }
  block_multisplit(dig, pos, S.wcount, S.dstart, S.tmp);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    if (dig[i] != NODIGIT) {
      S.K[src ^ 1][pos[i]] = kr[i];
      S.H[src ^ 1][pos[i]] = hr[i];
      if (WITH_G) S.G[src ^ 1][pos[i]] = gg[i];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(BLOCK) void k_local(const Seg *__restrict__ chunks, const uint64_t *__restrict__ keys0,
                                                 const uint64_t *__restrict__ keys1, const uint32_t *__restrict__ hdl0,
                                                 const uint32_t *__restrict__ hdl1, const uint64_t *__restrict__ packed,
                                                 const uint64_t *__restrict__ endbits, const uint64_t *__restrict__ offsets,
                                                 uint64_t n, uint64_t nb, uint32_t rmax, uint8_t *__restrict__ bwt,
                                                 uint64_t *__restrict__ term_pos, uint32_t *status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  LocalSmem &S = *reinterpret_cast<LocalSmem *>(smem_raw);
  const Seg ch = chunks[blockIdx.x];
  const uint32_t m = (uint32_t)ch.len;
  const uint64_t *Kg = ch.buf ? keys1 : keys0;
  const uint32_t *Hg = ch.buf ? hdl1 : hdl0;
  for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
    S.K[0][j] = Kg[ch.start + j];
    S.H[0][j] = Hg[ch.start + j];
  }
  __syncthreads();
  int cur = 0;
  // sort by the digits d..7 that vary inside the chunk (least significant first)
  {
    uint64_t o = 0, a = ~0ull;
    for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
      o |= S.K[0][j];
      a &= S.K[0][j];
    }
    o = block_or(o, S.tmp64);
    a = block_and(a, S.tmp64);
    const uint64_t diff = (o ^ a) & ~7ull;
    for (int j = 7; j >= (int)ch.d; --j) {
      if (diff & digit_mask(j)) {
        lds_pass<false>(S, cur, m, j);
        cur ^= 1;
      }
    }
  }
  // refinement of ties, window by window
  for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
    S.head[j] = (j == 0) || (order_bits(S.K[cur][j]) != order_bits(S.K[cur][j - 1]));
    S.fin[j] = 0;
  }
  __syncthreads();
  uint32_t r = ch.r;
  for (;;) {
    // group ranks (inclusive count of heads - 1) and group starts
    {
      const uint32_t base = threadIdx.x * ITEMS;
      uint32_t cnt = 0;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = base + i;
        if (j < m) cnt += S.head[j];
      }
      uint32_t total;
      uint32_t pre = block_excl_sum(cnt, S.scan_tmp, &total);
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = base + i;
        if (j < m) {
          pre += S.head[j];
          S.gr[j] = (uint16_t)(pre - 1);
          if (S.head[j]) S.hp[pre - 1] = (uint16_t)j;
        }
      }
      if (threadIdx.x == 0) S.hp[total] = (uint16_t)m;  // m <= CHUNK fits when CHUNK <= 65535
    }
    __syncthreads();
    uint32_t live_max = 0;
    for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
      if (S.fin[j]) continue;
      const uint32_t g = S.gr[j];
      const uint32_t a = S.hp[g], e = S.hp[g + 1];
      if (e - a == 1 || clamp_of(S.K[cur][a]) < (uint32_t)W) S.fin[j] = 1;
      else live_max = max(live_max, e - a);
    }
    live_max = block_max(live_max, S.tmp);
    if (live_max == 0) break;
    if (r + 1 > rmax) {
      if (threadIdx.x == 0) atomicOr(status, ST_WINDOW_BOUND);
      break;
    }
    ++r;
    // fetch the next window of every live suffix
    for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
      if (S.fin[j]) continue;
      const uint64_t k = S.K[cur][j];
      S.K[cur][j] = window_key(packed, endbits, nb, S.H[cur][j], r, (uint32_t)k & 7u);
    }
    __syncthreads();
    if (live_max <= (uint32_t)RANK_COUNT_MAX) {
      // stable rank inside each live group by all-pairs comparison
      for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
        const uint64_t kj = S.K[cur][j];
        if (S.fin[j]) {
          S.K[cur ^ 1][j] = kj;
          S.H[cur ^ 1][j] = S.H[cur][j];
          continue;
        }
        const uint32_t g = S.gr[j];
        const uint32_t a = S.hp[g], e = S.hp[g + 1];
        const uint64_t oj = order_bits(kj);
        uint32_t c = 0;
        for (uint32_t t = a; t < e; ++t) {
          const uint64_t ot = order_bits(S.K[cur][t]);
          c += (ot < oj) || (ot == oj && t < j);
        }
        S.K[cur ^ 1][a + c] = kj;
        S.H[cur ^ 1][a + c] = S.H[cur][j];
      }
      __syncthreads();
      cur ^= 1;
    } else {
      // composite stable LSD: new key digits, then the group start
      for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
        S.G[cur][j] = S.hp[S.gr[j]];
        if (S.fin[j]) S.K[cur][j] &= 7ull;  // final groups keep their place
      }
      __syncthreads();
      uint64_t o = 0, a = ~0ull;
      for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
        o |= S.K[cur][j];
        a &= S.K[cur][j];
      }
      o = block_or(o, S.tmp64);
      a = block_and(a, S.tmp64);
      const uint64_t diff = (o ^ a) & ~7ull;
      for (int jd = 7; jd >= 0; --jd) {
        if (diff & digit_mask(jd)) {
          lds_pass<true>(S, cur, m, jd);
          cur ^= 1;
        }
      }
      lds_pass<true>(S, cur, m, 8);
      cur ^= 1;
      lds_pass<true>(S, cur, m, 9);
      cur ^= 1;
    }
    // new group heads inside live groups
    for (uint32_t j = threadIdx.x; j < m; j += BLOCK) {
      if (S.fin[j]) continue;
      const uint32_t a = S.hp[S.gr[j]];
      if (j > a && order_bits(S.K[cur][j]) != order_bits(S.K[cur][j - 1])) S.head[j] = 1;
    }
    __syncthreads();
  }
  // a4: emit
  for (uint32_t j = threadIdx.x; j < m; j += BLOCK)
    emit_row(n + ch.start + j, S.K[cur][j], S.H[cur][j], offsets, n, bwt, term_pos);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
thread_local cxbwt_stats g_stats;

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t align_up(uint64_t x) { return (x + 255) & ~255ull; }

struct Layout {
  uint64_t keys0, keys1, hdl0, hdl1, endbits, tile_hist, segs, tile_prefix, seg_or, seg_and, seg_split, big_next,
      chunks, finals, counters, total;
  uint64_t cap_big, cap_chunks, cap_finals, max_tiles, endbit_words;
};

bool sizes_ok(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len) {
  return n_reads >= 1 && n_reads < (1ull << 32) && n_bases <= CXBWT_MAX_BASES && max_read_len <= CXBWT_MAX_READ_LEN;
}

Layout make_layout(uint64_t n_reads, uint64_t nb, uint32_t maxlen) {
  (void)n_reads;
  Layout L{};
  const uint64_t windows = (uint64_t)maxlen / W + 2;
  L.cap_big = nb / (CHUNK + 1) + 2;
  L.cap_finals = L.cap_big;
  // every chunk but the last of a run holds more than CHUNK/2 suffixes on
  // average with its successor; runs end at a big bucket or a parent's end
  L.cap_chunks = 2 * ceil_div(nb, CHUNK) + 2 * (8 * windows + 1) * L.cap_big + 2;
  L.max_tiles = ceil_div(nb, TILE) + L.cap_big + 1;
  L.endbit_words = nb / 64 + 2;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.keys0 = take(8 * nb);
  L.keys1 = take(8 * nb);
  L.hdl0 = take(4 * nb);
  L.hdl1 = take(4 * nb);
  L.endbits = take(8 * L.endbit_words);
  L.tile_hist = take(4 * 256 * L.max_tiles);
  L.segs = take(sizeof(Seg) * L.cap_big);
  L.tile_prefix = take(4 * (L.cap_big + 1));
  L.seg_or = take(8 * L.cap_big);
  L.seg_and = take(8 * L.cap_big);
  L.seg_split = take(L.cap_big);
  L.big_next = take(sizeof(Seg) * L.cap_big);
  L.chunks = take(sizeof(Seg) * L.cap_chunks);
  L.finals = take(sizeof(Seg) * L.cap_finals);
  L.counters = take(64);
  L.total = off;
  return L;
}

#define CX_CHECK(x)                                  \
  do {                                               \
    if ((x) != hipSuccess) return CXBWT_EDEVICE;     \
  } while (0)
#define CX_LAUNCHED()                                \
  do {                                               \
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

// counters block layout (uint32 slots)
enum { C_STATUS = 0, C_NBIG = 1, C_NCHUNK = 2, C_NFINAL = 3, C_COUNT = 16 };

int run_build(const uint64_t *packed, const uint64_t *offsets, uint64_t n, uint64_t nb, uint32_t maxlen, uint8_t *bwt,
              uint64_t *term_pos, unsigned char *ws, hipStream_t st) {
  g_stats = cxbwt_stats{};
  const Layout Lo = make_layout(n, nb, maxlen);
  uint64_t *keys0 = (uint64_t *)(ws + Lo.keys0);
  uint64_t *keys1 = (uint64_t *)(ws + Lo.keys1);
  uint32_t *hdl0 = (uint32_t *)(ws + Lo.hdl0);
  uint32_t *hdl1 = (uint32_t *)(ws + Lo.hdl1);
  uint64_t *endbits = (uint64_t *)(ws + Lo.endbits);
  uint32_t *tile_hist = (uint32_t *)(ws + Lo.tile_hist);
  Seg *segs = (Seg *)(ws + Lo.segs);
  uint32_t *tile_prefix = (uint32_t *)(ws + Lo.tile_prefix);
  unsigned long long *seg_or = (unsigned long long *)(ws + Lo.seg_or);
  unsigned long long *seg_and = (unsigned long long *)(ws + Lo.seg_and);
  uint8_t *seg_split = (uint8_t *)(ws + Lo.seg_split);
  Seg *big_next = (Seg *)(ws + Lo.big_next);
  Seg *chunks = (Seg *)(ws + Lo.chunks);
  Seg *finals = (Seg *)(ws + Lo.finals);
  uint32_t *counters = (uint32_t *)(ws + Lo.counters);
  const uint32_t rmax = maxlen / W + 1;

  int rc;
  if ((rc = fill_u32(counters, C_COUNT, 0, st))) return rc;
  if ((rc = fill_u64(endbits, Lo.endbit_words, 0, st))) return rc;
  k_prep<<<grid_for(n, 256), 256, 0, st>>>(packed, offsets, n, nb, maxlen, (unsigned long long *)endbits, bwt, term_pos,
                                          counters + C_STATUS);
  CX_LAUNCHED();
  uint32_t hc[C_COUNT];
  CX_CHECK(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, st));
  CX_CHECK(hipStreamSynchronize(st));
  if (hc[C_STATUS] & (ST_BAD_OFFSETS | ST_TOO_LONG)) return CXBWT_EDATA;
  if (nb == 0) return CXBWT_OK;

  k_gen<<<grid_for(nb, BLOCK), BLOCK, 0, st>>>(packed, endbits, nb, keys0, hdl0);
  CX_LAUNCHED();

  Lists Ls{big_next, counters + C_NBIG, (uint32_t)Lo.cap_big, chunks, counters + C_NCHUNK, (uint32_t)Lo.cap_chunks,
           finals, counters + C_NFINAL, (uint32_t)Lo.cap_finals, counters + C_STATUS, rmax};
  std::vector<Seg> big;
  uint32_t n_chunks = 0;
  if (nb > (uint64_t)CHUNK) {
    big.push_back(Seg{0, nb, 0, 0, 0, 0, 0});
  } else {
    Seg one{0, nb, 0, 0, 0, 0, 0};
    CX_CHECK(hipMemcpyAsync(chunks, &one, sizeof(Seg), hipMemcpyHostToDevice, st));
    n_chunks = 1;
  }
  std::vector<uint32_t> tprefix;
  while (!big.empty()) {
    const uint32_t ns = (uint32_t)big.size();
    if (ns > Lo.cap_big) return CXBWT_EDEVICE;
    tprefix.assign(ns + 1, 0);
    for (uint32_t i = 0; i < ns; ++i) tprefix[i + 1] = tprefix[i] + (uint32_t)ceil_div(big[i].len, TILE);
    const uint32_t ntiles = tprefix[ns];
    if (ntiles > Lo.max_tiles) return CXBWT_EDEVICE;
    CX_CHECK(hipMemcpyAsync(segs, big.data(), sizeof(Seg) * ns, hipMemcpyHostToDevice, st));
    CX_CHECK(hipMemcpyAsync(tile_prefix, tprefix.data(), 4 * (ns + 1), hipMemcpyHostToDevice, st));
    if ((rc = fill_u64((uint64_t *)seg_or, ns, 0, st))) return rc;
    if ((rc = fill_u64((uint64_t *)seg_and, ns, ~0ull, st))) return rc;
    if ((rc = fill_u32(counters + C_NBIG, 1, 0, st))) return rc;
    k_level_hist<<<ntiles, BLOCK, 0, st>>>(segs, tile_prefix, ns, keys0, keys1, hdl0, hdl1, packed, endbits, nb,
                                           tile_hist, seg_or, seg_and);
    CX_LAUNCHED();
    k_level_scan<<<ns, BLOCK, 0, st>>>(segs, tile_prefix, tile_hist, seg_or, seg_and, seg_split, Ls);
    CX_LAUNCHED();
    k_level_scatter<<<ntiles, BLOCK, 0, st>>>(segs, tile_prefix, ns, seg_split, tile_hist, keys0, keys1, hdl0, hdl1);
    CX_LAUNCHED();
    CX_CHECK(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, st));
    CX_CHECK(hipStreamSynchronize(st));
    if (hc[C_STATUS]) return CXBWT_EDEVICE;
    g_stats.levels++;
    g_stats.big_segments += ns;
    const uint32_t nn = hc[C_NBIG];
    big.resize(nn);
    if (nn) {
      CX_CHECK(hipMemcpyAsync(big.data(), big_next, sizeof(Seg) * nn, hipMemcpyDeviceToHost, st));
      CX_CHECK(hipStreamSynchronize(st));
      for (const Seg &s : big) g_stats.max_window = std::max(g_stats.max_window, s.r);
    }
    n_chunks = hc[C_NCHUNK];
  }
  if (n_chunks) {
    const size_t smem = sizeof(LocalSmem);
    k_local<<<n_chunks, BLOCK, smem, st>>>(chunks, keys0, keys1, hdl0, hdl1, packed, endbits, offsets, n, nb, rmax,
                                           bwt, term_pos, counters + C_STATUS);
    CX_LAUNCHED();
  }
  g_stats.chunks = n_chunks;
  const uint32_t nfin = hc[C_NFINAL];
  if (nfin) {
    std::vector<Seg> fin(nfin);
    CX_CHECK(hipMemcpyAsync(fin.data(), finals, sizeof(Seg) * nfin, hipMemcpyDeviceToHost, st));
    CX_CHECK(hipStreamSynchronize(st));
    tprefix.assign(nfin + 1, 0);
    for (uint32_t i = 0; i < nfin; ++i) tprefix[i + 1] = tprefix[i] + (uint32_t)ceil_div(fin[i].len, TILE);
    CX_CHECK(hipMemcpyAsync(tile_prefix, tprefix.data(), 4 * (nfin + 1), hipMemcpyHostToDevice, st));
    k_emit_final<<<tprefix[nfin], BLOCK, 0, st>>>(finals, tile_prefix, nfin, keys0, keys1, hdl0, hdl1, offsets, n, bwt,
                                                  term_pos);
    CX_LAUNCHED();
  }
  g_stats.final_big = nfin;
  CX_CHECK(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, st));
  CX_CHECK(hipStreamSynchronize(st));
  if (hc[C_STATUS]) return CXBWT_EDEVICE;
  return CXBWT_OK;
}

bool local_smem_configured = false;

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
  return (size_t)make_layout(n_reads, n_bases, max_read_len).total;
}

int cxbwt_build(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                uint32_t max_read_len, uint8_t *bwt, uint64_t *term_pos, void *workspace, size_t workspace_bytes,
                void *stream) {
  if (!packed || !offsets || !bwt || !term_pos || !workspace || n_reads == 0) return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (workspace_bytes < cxbwt_workspace_bytes(n_reads, n_bases, max_read_len)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  if (!local_smem_configured) {
    // raise the dynamic LDS limit where the runtime asks for it; a launch
    // that still does not fit reports an error through hipGetLastError
    (void)hipFuncSetAttribute((const void *)k_local, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)sizeof(LocalSmem));
    local_smem_configured = true;
  }
  return run_build(packed, offsets, n_reads, n_bases, max_read_len, bwt, term_pos, (unsigned char *)workspace,
                   (hipStream_t)stream);
}

int cxbwt_last_stats(cxbwt_stats *out) {
  if (!out) return CXBWT_EINVAL;
  *out = g_stats;
  return CXBWT_OK;
}

const char *cxbwt_status_str(int status) {
  switch (status) {
    case CXBWT_OK: return "ok";
    case CXBWT_EINVAL: return "invalid argument (null pointer or inconsistent sizes)";
    case CXBWT_ERANGE: return "size out of the supported range";
    case CXBWT_ENOMEM: return "workspace smaller than cxbwt_workspace_bytes()";
    case CXBWT_EDEVICE: return "HIP launch/runtime failure or internal device check failed";
    case CXBWT_EDATA: return "invalid input data found on the device (offsets, read length or bases)";
    default: return "unknown status";
  }
}

}  // extern "C"
