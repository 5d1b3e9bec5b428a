// Host build of the library's window-key functions (device_common.h) for a
// CPU test: the functions are __host__ __device__, so compiled host-only they
// are the same code the kernels run.  The test builds text records from their
// documented layout in Python and compares these keys with a per-base
// construction of (bases zero-padded past the read end, clamped length,
// preceding symbol).
#include "device_common.h"

extern "C" uint64_t wk_first_key(const void *text, uint64_t nb, uint64_t p) {
  return cxk::first_key(static_cast<const cxk::TextRec *>(text), nb, p);
}

extern "C" uint64_t wk_window_key(const void *text, uint64_t nb, uint64_t p, uint32_t r, uint32_t prev3) {
  return cxk::window_key(static_cast<const cxk::TextRec *>(text), nb, p, r, prev3);
}

extern "C" uint32_t wk_window() { return (uint32_t)cxk::W; }
