// ceilings.hip -- a measurement kernel for bench.py's memory-system ceilings,
// built into its own library (libcxbwt_ceilings.so), apart from the BWT
// library.  It gathers rows at hashed random indices from a table in device
// memory, as the chunk kernel's window loads do: 16-byte rows (one record a
// window) or 32-byte rows (an aligned pair of 16-byte loads).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// splitmix64 finaliser (Steele, Lea and Flood): a well-spread row index per
// load index
__device__ __forceinline__ uint64_t spread(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

constexpr int GATHER_BATCH = 4;  // loads in flight per thread

template <int PAIR>
__global__ __launch_bounds__(256) void k_gather(const uint4 *__restrict__ table, uint64_t row_mask, uint64_t n,
                                                uint64_t seed, uint32_t *__restrict__ sink) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (uint64_t i0 = tid; i0 < n; i0 += nth * GATHER_BATCH) {
    uint4 a[GATHER_BATCH], b[GATHER_BATCH];
#pragma unroll
    for (int k = 0; k < GATHER_BATCH; ++k) {
      const uint64_t i = i0 + (uint64_t)k * nth;
      if (i < n) {
        const uint64_t r = spread(seed ^ i) & row_mask;
        a[k] = table[PAIR ? 2 * r : r];
        if (PAIR) b[k] = table[2 * r + 1];
      }
    }
#pragma unroll
    for (int k = 0; k < GATHER_BATCH; ++k) {
      const uint64_t i = i0 + (uint64_t)k * nth;
      if (i < n) acc ^= a[k].x ^ a[k].w ^ (PAIR ? (b[k].y ^ b[k].z) : 0u);
    }
  }
  // a data-dependent store keeps every load
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

}  // namespace

// n gathers of row_bytes (16 or 32) bytes at random rows of a table of rows
// rows (a power of two; the table holds rows * row_bytes bytes, 16-byte
// aligned), enqueued on stream.  Returns 0, or -1 for invalid arguments,
// -4 for a launch error.  sink: one uint32 of device memory the kernel may
// write.
extern "C" int cxbwt_ceiling_gather(const void *table, uint64_t rows, uint32_t row_bytes, uint64_t n, uint64_t seed,
                                    uint32_t *sink, void *stream) {
  if (!table || !sink || rows == 0 || (rows & (rows - 1)) != 0 || (row_bytes != 16 && row_bytes != 32) ||
      ((uintptr_t)table & 15u) != 0)
    return -1;
  const hipStream_t st = (hipStream_t)stream;
  const unsigned grid = 256 * 16, block = 256;
  if (row_bytes == 16)
    k_gather<0><<<grid, block, 0, st>>>((const uint4 *)table, rows - 1, n, seed, sink);
  else
    k_gather<1><<<grid, block, 0, st>>>((const uint4 *)table, rows - 1, n, seed, sink);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
