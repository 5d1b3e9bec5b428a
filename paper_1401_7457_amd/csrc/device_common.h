// device_common.h -- key layout, window fetch and workgroup primitives shared
// by the kernels of cxbwt.hip (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cxk {

constexpr int W = 28;              // bases per key window
constexpr int BLOCK = 256;         // threads per workgroup
constexpr int WAVES = BLOCK / 64;  // wave64
constexpr uint32_t NODIGIT = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Suffix key of one 28-base window (see cxbwt.hip for why this order is the
// suffix order):
//   bits 63..8  the 28 bases, 2 bits each, first base highest; zero past the
//               end of the read
//   bits  7..3  clamped length: min(bases left in the read from the window
//               start, 28)
//   bits  2..0  symbol preceding the suffix: 0..3 = A,C,G,T, 4 = '$'
// Only bits [3, 64) take part in comparisons.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t order_bits(uint64_t k) { return k & ~7ull; }
__device__ __forceinline__ uint32_t clamp_of(uint64_t k) { return (uint32_t)(k >> 3) & 31u; }
// 8-bit digit j (0 = most significant) of the ordering bits; digit 7 is the
// 5-bit clamped length
__device__ __forceinline__ uint32_t digit_of(uint64_t k, int j) {
  return j < 7 ? (uint32_t)(k >> (56 - 8 * j)) & 0xFFu : (uint32_t)(k >> 3) & 0x1Fu;
}
__host__ __device__ __forceinline__ uint64_t digit_mask(int j) {
  return j < 7 ? (0xFFull << (56 - 8 * j)) : (0x1Full << 3);
}
// ---------------------------------------------------------------------------
// Text records: the 2-bit bases interleaved with read-start bits, 16 bytes
// per 32 bases, so that one window of any suffix is a single 32-byte read.
//   bases   32 bases, first base in the top two bits (the packed input word)
//   starts  bit t set when base 32*w + t is the first base of a non-empty
//           read; one extra start bit marks position B (the end of the text)
// A record array holds ceil(B/32) + 2 records; the last ones are padding.
// ---------------------------------------------------------------------------
struct alignas(16) TextRec {
  uint64_t bases;
  uint32_t starts;
  uint32_t pad;
};

__device__ __forceinline__ uint32_t rec_base(const TextRec *__restrict__ text, uint64_t t) {
  return (uint32_t)(text[t >> 5].bases >> (62 - 2 * (t & 31))) & 3u;
}
__device__ __forceinline__ bool rec_start(const TextRec *__restrict__ text, uint64_t t) {
  return (text[t >> 5].starts >> (t & 31)) & 1u;
}

// The two records a window key is built from, loaded before use so many
// windows can be in flight per thread.  The record index is clamped into the
// array (a clamped read is never used).
struct WinWords {
  TextRec a, b;
};

__device__ __forceinline__ WinWords window_load(const TextRec *__restrict__ text, uint64_t nb, uint64_t p,
                                                uint32_t r) {
  const uint64_t q = p + (uint64_t)W * r;
  const uint64_t qc = q <= nb ? q : nb;
  WinWords w;
  w.a = text[qc >> 5];
  w.b = text[(qc >> 5) + 1];
  return w;
}

// Key of window r of the suffix starting at base p (the window starts at
// q = p + 28 r).  The suffix's read ends just before the first read start s
// after p; the window holds min(s - q, 28) bases.  For r >= 1 the suffix is
// live: its read holds at least 28 r bases from p, so s >= q.
__device__ __forceinline__ uint64_t window_combine(const WinWords &w, uint64_t nb, uint64_t p, uint32_t r,
                                                   uint32_t prev3) {
  const uint64_t q = p + (uint64_t)W * r;
  if (q > nb) return prev3;  // never taken for a live suffix
  const uint64_t lo = r == 0 ? p + 1 : q;          // first position a start may sit at
  const uint32_t o = (uint32_t)(lo - ((q >> 5) << 5));  // 0..32, offset of lo in the record pair
  const uint64_t st = ((uint64_t)w.b.starts << 32) | w.a.starts;
  const uint64_t from = o < 64 ? st >> o : 0ull;
  const uint64_t s_rel = from ? (uint64_t)o + (uint64_t)__builtin_ctzll(from) : ~0ull;  // start - 32*(q>>5)
  const uint64_t q_rel = q & 31;
  const uint32_t clamp = (s_rel != ~0ull && s_rel < q_rel + W) ? (uint32_t)(s_rel - q_rel) : (uint32_t)W;
  uint64_t chars = 0;
  if (clamp > 0) {
    const uint32_t b = 2u * (uint32_t)q_rel;
    uint64_t x = w.a.bases << b;
    if (b) x |= w.b.bases >> (64 - b);
    chars = x & ~0xFFull;
    if (clamp < (uint32_t)W) chars &= ~((1ull << (64 - 2 * clamp)) - 1);
  }
  return chars | ((uint64_t)clamp << 3) | prev3;
}

__device__ __forceinline__ uint64_t window_key(const TextRec *__restrict__ text, uint64_t nb, uint64_t p, uint32_t r,
                                               uint32_t prev3) {
  return window_combine(window_load(text, nb, p, r), nb, p, r, prev3);
}

// Window-0 key of the suffix starting at base p, with its preceding symbol:
// '$' when p starts a read, else base p-1.
__device__ __forceinline__ uint64_t first_key(const TextRec *__restrict__ text, uint64_t nb, uint64_t p) {
  const WinWords w = window_load(text, nb, p, 0);
  uint32_t prev3 = 4;
  if (!((w.a.starts >> (p & 31)) & 1u)) prev3 = rec_base(text, p - 1);
  return window_combine(w, nb, p, 0, prev3);
}

// ---------------------------------------------------------------------------
// wave / workgroup primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
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
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *tmp, uint32_t *total) {
  const uint32_t inc = wave_incl_sum(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) tmp[w] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) {
    const uint32_t x = tmp[i];
    if (i < w) pre += x;
    tot += x;
  }
  __syncthreads();
  if (total) *total = tot;
  return pre + inc - v;
}

__device__ __forceinline__ uint64_t block_or(uint64_t v, uint64_t *tmp) {
  v = wave_or(v);
  if (lane_id() == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) r |= tmp[i];
  __syncthreads();
  return r;
}
__device__ __forceinline__ uint64_t block_and(uint64_t v, uint64_t *tmp) {
  v = wave_and(v);
  if (lane_id() == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = ~0ull;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) r &= tmp[i];
  __syncthreads();
  return r;
}
__device__ __forceinline__ uint32_t block_max(uint32_t v, uint32_t *tmp) {
  v = wave_max(v);
  if (lane_id() == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) r = max(r, tmp[i]);
  __syncthreads();
  return r;
}

// Position of item i of this thread when a workgroup holds NI items per
// thread: wave w owns [w*64*NI, (w+1)*64*NI); item i of lane l sits at
// w*64*NI + i*64 + l (consecutive lanes touch consecutive elements).
template <int NI>
__device__ __forceinline__ uint32_t item_index(int i) {
  return (uint32_t)((threadIdx.x >> 6) * (64 * NI) + i * 64) + lane_id();
}

// Stable 256-way split of up to BLOCK*NI items held in registers (layout of
// item_index<NI>).  On return pos[i] is the destination of item i in
// [0, count) and dstart[d] the first destination of digit d.  dig[i] ==
// NODIGIT marks an absent item.  Ranks inside a wave come from ballot-matched
// peer masks; waves are ordered by a digit-major scan of per-wave counts.
template <int NI>
__device__ __forceinline__ void block_multisplit(const uint32_t (&dig)[NI], uint32_t (&pos)[NI], uint32_t *wcount,
                                                 uint32_t *dstart, uint32_t *tmp) {
  const int w = threadIdx.x >> 6;
  for (int x = threadIdx.x; x < WAVES * 256; x += BLOCK) wcount[x] = 0;
  __syncthreads();
  uint32_t *wc = wcount + w * 256;
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int i = 0; i < NI; ++i) {
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
  const uint32_t d = threadIdx.x;  // one digit per thread (BLOCK == 256)
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
  for (int i = 0; i < NI; ++i)
    if (dig[i] != NODIGIT) pos[i] += dstart[dig[i]] + wc[dig[i]];
}

static_assert(BLOCK == 256, "block_multisplit assigns one digit per thread");

}  // namespace cxk
