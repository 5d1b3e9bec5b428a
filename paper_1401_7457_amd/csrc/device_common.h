// device_common.h -- key layout, window fetch and workgroup primitives shared
// by the kernels of cxbwt.hip (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cxk {

constexpr int W = 27;              // bases per key window
constexpr int BLOCK = 256;         // threads per workgroup
constexpr int WAVES = BLOCK / 64;  // wave64
constexpr uint32_t NODIGIT = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// Suffix key of one 27-base window (see cxbwt.hip for why this order is the
// suffix order):
//   bits 63..10 the 27 bases, 2 bits each, first base highest; zero past the
//               end of the read
//   bits  9..8  zero
//   bits  7..3  clamped length: min(bases left in the read from the window
//               start, 27)
//   bits  2..0  symbol preceding the suffix: 0..3 = A,C,G,T, 4 = '$'
// Only bits [3, 64) take part in comparisons.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t order_bits(uint64_t k) { return k & ~7ull; }
__host__ __device__ __forceinline__ uint32_t clamp_of(uint64_t k) { return (uint32_t)(k >> 3) & 31u; }
// 8-bit digit j (0 = most significant) of the ordering bits; digit 7 is the
// 5-bit clamped length
__host__ __device__ __forceinline__ uint32_t digit_of(uint64_t k, int j) {
  return j < 7 ? (uint32_t)(k >> (56 - 8 * j)) & 0xFFu : (uint32_t)(k >> 3) & 0x1Fu;
}
__host__ __device__ __forceinline__ uint64_t digit_mask(int j) {
  return j < 7 ? (0xFFull << (56 - 8 * j)) : (0x1Full << 3);
}
// ---------------------------------------------------------------------------
// Text records: one 16-byte record per 16 bases, each holding everything a
// window starting in its 16 positions needs, so a window is one aligned
// 16-byte load.  Record w covers positions 16w .. 16w+41:
//   hi  bits 63..0   bases 16w .. 16w+31, first base in the top two bits
//   lo  bits 63..44  bases 16w+32 .. 16w+41, same order
//       bits 43..42  base 16w-1 (zero for w = 0)
//       bits 41..0   start bits: bit k set when position 16w+k is the first
//                    base of a non-empty read, or k = B - 16w (the end of the
//                    text, B bases in all)
// 3 bits per position: 42 positions fit 126 bits, enough for a window of
// 27 bases starting at any of the 16 (15 + 27 = 42).  A record array holds
// floor(B/16) + 2 records; positions past B read as zero.
// ---------------------------------------------------------------------------
struct alignas(16) TextRec {
  uint64_t hi;
  uint64_t lo;
};

constexpr int REC_SPAN = 42;                             // positions per record
constexpr uint64_t REC_STARTS = (1ull << REC_SPAN) - 1;  // start-bit field of lo

// base at offset k (0..41) of a record
__host__ __device__ __forceinline__ uint32_t rec_base_at(const TextRec &t, uint32_t k) {
  return k < 32 ? (uint32_t)(t.hi >> (62 - 2 * k)) & 3u : (uint32_t)(t.lo >> (62 - 2 * (k - 32))) & 3u;
}

// The record a window starting at q is built from, loaded before use so many
// windows can be in flight per thread.  q is clamped to B (a clamped read is
// never used).
__host__ __device__ __forceinline__ TextRec window_load(const TextRec *__restrict__ text, uint64_t nb, uint64_t p, uint32_t r) {
  const uint64_t q = p + (uint64_t)W * r;
  const uint64_t qc = q <= nb ? q : nb;
  return text[qc >> 4];
}

// Key of window r of the suffix starting at base p (the window starts at
// q = p + 27 r).  The suffix's read ends just before the first read start s
// after p; the window holds min(s - q, 27) bases.  For r >= 1 the suffix is
// live: its read holds at least 27 r bases from p, so s >= q.
__host__ __device__ __forceinline__ uint64_t window_combine(const TextRec &t, uint64_t nb, uint64_t p, uint32_t r,
                                                   uint32_t prev3) {
  const uint64_t q = p + (uint64_t)W * r;
  if (q > nb) return prev3;  // never taken for a live suffix
  const uint32_t o = (uint32_t)(q & 15);      // window start inside the record
  const uint32_t lo_off = r == 0 ? o + 1 : o;  // first position a start may sit at
  const uint64_t from = (t.lo & REC_STARTS) >> lo_off;
  const uint32_t s_rel = from ? lo_off + (uint32_t)__builtin_ctzll(from) : 64u;
  const uint32_t clamp = s_rel < o + (uint32_t)W ? s_rel - o : (uint32_t)W;
  uint64_t chars = 0;
  if (clamp > 0) {
    uint64_t x = t.hi << (2 * o);
    if (o) x |= t.lo >> (64 - 2 * o);
    chars = x & ~0x3FFull;
    if (clamp < (uint32_t)W) chars &= ~((1ull << (64 - 2 * clamp)) - 1);
  }
  return chars | ((uint64_t)clamp << 3) | prev3;
}

__host__ __device__ __forceinline__ uint64_t window_key(const TextRec *__restrict__ text, uint64_t nb, uint64_t p, uint32_t r,
                                               uint32_t prev3) {
  return window_combine(window_load(text, nb, p, r), nb, p, r, prev3);
}

// Window-0 key of the suffix starting at base p, with its preceding symbol:
// '$' when p starts a read, else base p-1; t is the record of p (text[p/16]).
__host__ __device__ __forceinline__ uint64_t first_key_from(const TextRec &t, uint64_t nb, uint64_t p) {
  const uint32_t o = (uint32_t)(p & 15);
  uint32_t prev3 = 4;
  if (!((t.lo >> o) & 1u)) prev3 = o ? rec_base_at(t, o - 1) : (uint32_t)(t.lo >> 42) & 3u;
  return window_combine(t, nb, p, 0, prev3);
}

__host__ __device__ __forceinline__ uint64_t first_key(const TextRec *__restrict__ text, uint64_t nb, uint64_t p) {
  return first_key_from(window_load(text, nb, p, 0), nb, p);
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

// Exclusive prefix sum of one value per thread over a workgroup of NW waves.
template <int NW = WAVES>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t v, uint32_t *tmp, uint32_t *total) {
  const uint32_t inc = wave_incl_sum(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) tmp[w] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
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

// The lanes among `live` whose 8-bit value d equals this lane's: one ballot
// per bit, each lane keeping the lanes that agree with its own bit.  The bit
// is sign-extended to a 32-bit mask t (all ones when set), so the agreeing
// lanes are ~(ballot ^ t), one three-input bit operation per mask half.
__device__ __forceinline__ uint64_t wave_match8(uint32_t d, uint64_t live) {
  uint32_t lo = (uint32_t)live, hi = (uint32_t)(live >> 32);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint32_t t = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
    const uint64_t v = __ballot(t != 0u);
    lo &= ~((uint32_t)v ^ t);
    hi &= ~((uint32_t)(v >> 32) ^ t);
  }
  return ((uint64_t)hi << 32) | lo;
}

// Stable 256-way split of up to 64*NW*NI items held in registers by a
// workgroup of NW waves (layout of item_index<NI>).  On return pos[i] is the
// destination of item i in [0, count) and dstart[d] the first destination of
// digit d.  dig[i] == NODIGIT marks an absent item.  Ranks inside a wave come
// from ballot-matched peer masks; waves are ordered by a digit-major scan of
// per-wave counts (wcount holds NW * 256 counters, tmp NW words).
template <int NI, int NW = WAVES>
__device__ __forceinline__ void block_multisplit(const uint32_t (&dig)[NI], uint32_t (&pos)[NI], uint32_t *wcount,
                                                 uint32_t *dstart, uint32_t *tmp) {
  static_assert(NW >= 4, "one digit per thread of the first four waves");
  const int w = threadIdx.x >> 6;
  for (int x = threadIdx.x; x < NW * 256; x += NW * 64) wcount[x] = 0;
  __syncthreads();
  uint32_t *wc = wcount + w * 256;
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const uint32_t d = dig[i];
    const bool valid = d != NODIGIT;
    const uint64_t peers = wave_match8(d, __ballot(valid));
    if (valid) {
      const uint32_t before = wc[d];
      pos[i] = before + (uint32_t)__popcll(peers & lt);
      if ((peers & lt) == 0) wc[d] = before + (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();
  const uint32_t d = threadIdx.x;  // one digit per thread of the first 256
  uint32_t run = 0;
  if (d < 256) {
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      const uint32_t c = wcount[ww * 256 + d];
      wcount[ww * 256 + d] = run;
      run += c;
    }
  }
  const uint32_t ex = block_excl_sum<NW>(run, tmp, nullptr);
  if (d < 256) dstart[d] = ex;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NI; ++i)
    if (dig[i] != NODIGIT) pos[i] += dstart[dig[i]] + wc[dig[i]];
}

static_assert(BLOCK == 256, "a default workgroup holds one thread per digit");

}  // namespace cxk
