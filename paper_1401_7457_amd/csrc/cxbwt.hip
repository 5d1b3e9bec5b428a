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
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "cxbwt.h"
#include "cxbwt_kernels.h"

namespace {

using namespace cxk;

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
thread_local cxbwt_stats g_stats;
thread_local int g_timing = 0;

// The instantiation a build uses (see the tuning constants).
struct Tuning {
  uint32_t tile_items;   // 6, 8 or 16 suffixes per 256 threads' thread in a level tile (16: 8 waves x 8)
  uint32_t chunk_items;  // 3, 6 or 8 suffixes per lane in a chunk
  uint32_t schedule = CXBWT_SCHEDULE_MSD;  // sort schedule of single-collection builds
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
      stats, list_tiles, list_blocks, ph_counts, ph_prefixes, pos64, total;
  uint64_t cap_big, cap_chunks, cap_finals, seg_slots, max_tiles, max_groups, n_rec, n_rank_words, n_rank_blocks;
  uint64_t sort_cap, n_cmap, n_list_tiles, n_list_blocks, tile_hist_bytes;
};

bool sizes_ok(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len) {
  return n_reads >= 1 && n_reads < (1ull << 32) && n_bases <= CXBWT_MAX_BASES && max_read_len <= CXBWT_MAX_READ_LEN;
}
// A build in ranges: the handles of one range are 32-bit (sort positions of
// at most max_range_suffixes suffixes), so the collection may exceed 32-bit
// base positions when they are kept in a 64-bit table.
bool range_wide(uint64_t n_bases, uint32_t flags) {
  return n_bases > CXBWT_MAX_BASES || (flags & CXBWT_RANGE_WIDE) != 0;
}
bool range_sizes_ok(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len, uint64_t m, uint32_t flags) {
  (void)flags;
  return n_reads >= 1 && n_reads < (1ull << 32) && n_bases <= CXBWT_MAX_RANGE_BASES &&
         max_read_len <= CXBWT_MAX_READ_LEN && m >= 1 && m <= CXBWT_MAX_BASES;
}

// Workspace of a build of nb bases in n_reads reads and n_coll collections
// whose sort buffers hold at most m_sort suffixes at once (all nb of them,
// or one range of a build in ranges).
Layout make_layout(uint64_t n_reads, uint64_t nb_text, uint32_t n_coll, uint64_t m_sort = ~0ull, bool wide = false) {
  Layout L{};
  const uint64_t nb = std::min(nb_text, m_sort);  // suffixes sorted at once
  L.sort_cap = nb;
  L.n_cmap = n_coll;  // a build in ranges rewrites its one entry per range
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
  L.n_rec = nb_text / 16 + 2;
  L.n_list_tiles = ceil_div(nb_text, LIST_TILE) + 1;
  L.n_list_blocks = ceil_div(L.n_list_tiles, RANK_BLOCK_WORDS) + 1;
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
  // the read-start bitmap (one bit per base) lives here before level 1
  L.tile_hist_bytes = std::max<uint64_t>(4 * 256 * L.max_tiles, 4 * (nb_text / 32 + 4));
  L.tile_hist = take(L.tile_hist_bytes);
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
  L.cmap = take(sizeof(CollMap) * L.n_cmap);
  L.counters = take(4 * C_COUNT);
  L.stats = take(8 * STAT_WORDS);
  L.list_tiles = take(4 * L.n_list_tiles);
  L.list_blocks = take(4 * L.n_list_blocks);
  L.ph_counts = take(8 * 256 * PH_MAX_PREFIXES);
  L.ph_prefixes = take(8 * PH_MAX_PREFIXES);
  // wide positions: a 64-bit position per listed suffix; 0 = no table (the
  // layout starts with keys0 at offset 0, so no other region sits there)
  L.pos64 = wide ? take(8 * nb) : 0;
  L.total = off;
  return L;
}

// The text behind the calling thread's last CXBWT_EDEVICE or CXBWT_EDATA
// (cxbwt_last_error).
thread_local char g_last_error[256] = "";
int fail_hip(hipError_t e, const char *what) {
  snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
  return CXBWT_EDEVICE;
}
// An internal size check that failed (a list or scratch area smaller than
// the work handed to it).
int fail_internal(const char *what) {
  snprintf(g_last_error, sizeof(g_last_error), "internal check failed: %s", what);
  return CXBWT_EDEVICE;
}

// A failure the device reported in its status word.
int fail_status(uint32_t status) {
  snprintf(g_last_error, sizeof(g_last_error), "device status 0x%x:%s%s%s%s%s%s", status,
           (status & ST_BAD_OFFSETS) ? " offsets are not a non-decreasing partition of the bases;" : "",
           (status & ST_TOO_LONG) ? " a read is longer than max_read_len;" : "",
           (status & ST_BAD_CHAR) ? " a byte is not A/C/G/T;" : "",
           (status & ST_LIST_OVERFLOW) ? " a work list overflowed its capacity;" : "",
           (status & ST_WINDOW_BOUND) ? " a tie outlived the windows of max_read_len;" : "",
           (status & ST_PLAN_MISMATCH) ? " collection bases differ from the captured plan;" : "");
  if (status & (ST_BAD_OFFSETS | ST_TOO_LONG)) return CXBWT_EDATA;
  if (status & ST_PLAN_MISMATCH) return CXBWT_EINVAL;
  return CXBWT_EDEVICE;
}

#define CX_CHECK(x)                                                        \
  do {                                                                     \
    const hipError_t cx_e_ = (x);                                          \
    if (cx_e_ != hipSuccess) return fail_hip(cx_e_, "HIP runtime call");   \
  } while (0)
#define CX_LAUNCHED()                                                      \
  do {                                                                     \
    const hipError_t cx_e_ = hipGetLastError();                            \
    if (cx_e_ != hipSuccess) return fail_hip(cx_e_, "kernel launch");      \
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
  uint64_t *keys0, *keys1, *start_row, *coll_reads, *coll_bases, *ph_prefixes;
  uint64_t *pos64;  // 64-bit positions of the listed range (wide builds in ranges), else null
  uint32_t *list_tiles, *list_blocks;
  unsigned long long *ph_counts;
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
  if (ns > Lo.seg_slots) return fail_internal("work exceeds a workspace list or scratch area");
  tprefix.assign(ns + 1, 0);
  gprefix.assign(ns + 1, 0);
  for (uint32_t i = 0; i < ns; ++i) {
    const uint32_t nt = (uint32_t)ceil_div(segs[i].len, tile_len);
    tprefix[i + 1] = tprefix[i] + nt;
    gprefix[i + 1] = gprefix[i] + (uint32_t)ceil_div(nt, GROUP_TILES);
  }
  ntiles = tprefix[ns];
  ngroups = gprefix[ns];
  if (ntiles > Lo.max_tiles || ngroups > Lo.max_groups) return fail_internal("work exceeds a workspace list or scratch area");
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
      k_local<LI, OCC, false><<<grid, LOCAL_WG, 0, st>>>(B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.pos64, B.text,\
                                                        B.srank, B.cmap, nb, rmax, bwt, B.start_row,             \
                                                        B.counters + C_STATUS, B.stats, 0, dev_nchunks, 0);      \
      k_local<LI, OCCP, true><<<256u, LOCAL_WG, 0, st>>>(B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.pos64, B.text,\
                                                        B.srank, B.cmap, nb, rmax, bwt, B.start_row,             \
                                                        B.counters + C_STATUS, B.stats, 0, dev_nchunks, grid);   \
    } else if (dev_nchunks) {                                                                                    \
      k_local<LI, OCCP, true><<<256u * 4u * OCCP, LOCAL_WG, 0, st>>>(                                            \
          B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.pos64, B.text, B.srank, B.cmap, nb, rmax, bwt, B.start_row,\
          B.counters + C_STATUS, B.stats, 0, dev_nchunks, 0);                                                    \
    } else {                                                                                                     \
      k_local<LI, OCC, false><<<n_chunks, LOCAL_WG, 0, st>>>(B.chunks, B.keys0, B.keys1, B.hdl0, B.hdl1, B.pos64, B.text,\
                                                            B.srank, B.cmap, nb, rmax, bwt, B.start_row,         \
                                                            B.counters + C_STATUS, B.stats, n_chunks, nullptr,   \
                                                            0);                                                  \
    }                                                                                                            \
  } while (0)
  // waves per SIMD the register allocation is held to: 8 per lane at 4, 6 per
  // lane at 6 (70 registers; the LDS of a 384-suffix chunk, 6.4 KB, also
  // allows six), 3 per lane at 7 (8 spills and is slower)
  if (tu.chunk_items == 8) CX_LOCAL(8, 4, 3);
  else if (tu.chunk_items == 6) CX_LOCAL(6, 6, 4);
  else CX_LOCAL(3, 7, 5);
#undef CX_LOCAL
  CX_LAUNCHED();
  return CXBWT_OK;
}

// Finish the chunks and final groups a level produced.
int finish_level(const Buffers &B, const Layout &Lo, const Tuning &tu, uint64_t nb, uint32_t rmax, uint8_t *bwt,
                 uint32_t n_chunks, uint32_t n_finals, uint64_t final_tiles, uint64_t final_len, PhaseTimer &T,
                 hipStream_t st) {
  if (n_chunks > Lo.cap_chunks || n_finals > Lo.cap_finals) return fail_internal("work exceeds a workspace list or scratch area");
  int rc;
  if (n_chunks) {
    T.begin();
    if ((rc = launch_local(B, tu, nb, rmax, bwt, n_chunks, nullptr, st))) return rc;
    T.end(PH_LOCAL);
    g_stats.chunks += n_chunks;
  }
  if (n_finals) {
    if (final_tiles == 0 || final_tiles > 0xFFFFFFFFull) return fail_internal("work exceeds a workspace list or scratch area");
    if ((rc = prefix_list(B, B.finals, n_finals, tu.tile_len(), nullptr, B.tile_prefix, nullptr, st))) return rc;
    T.begin();
    k_emit_final<false><<<(unsigned)final_tiles, BLOCK, 0, st>>>(B.finals, B.tile_prefix, n_finals, nullptr, tu.tile_len(),
                                                          B.keys0, B.keys1, B.hdl0, B.hdl1, B.pos64, B.text, B.srank,
                                                          B.cmap, bwt, B.start_row);
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
                                                                B.pos64, B.tile_hist, B.seg_or, B.seg_and)
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
  B.list_tiles = (uint32_t *)(ws + Lo.list_tiles);
  B.list_blocks = (uint32_t *)(ws + Lo.list_blocks);
  B.ph_counts = (unsigned long long *)(ws + Lo.ph_counts);
  B.ph_prefixes = (uint64_t *)(ws + Lo.ph_prefixes);
  B.pos64 = Lo.pos64 ? (uint64_t *)(ws + Lo.pos64) : nullptr;
  return B;
}

void build_init(Build &b, const uint64_t *packed, const uint64_t *offsets, uint64_t n, uint64_t nb, uint32_t maxlen,
                const uint64_t *coll_reads, uint32_t ncoll, uint8_t *bwt, uint64_t *term_pos, unsigned char *ws,
                uint64_t m_sort = ~0ull, bool wide = false) {
  b.packed = packed;
  b.offsets = offsets;
  b.n = n;
  b.nb = nb;
  b.maxlen = maxlen;
  b.ncoll = ncoll;
  b.bwt = bwt;
  b.term_pos = term_pos;
  b.Lo = make_layout(n, nb, ncoll, m_sort, wide);
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
  if (4 * n_sbits > b.Lo.tile_hist_bytes) return fail_internal("work exceeds a workspace list or scratch area");
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
  if (hc[C_STATUS] & (ST_BAD_OFFSETS | ST_TOO_LONG)) return fail_status(hc[C_STATUS]);
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
  if (s.ns > Lo.seg_slots || s.ntiles > Lo.max_tiles || s.ngroups > Lo.max_groups) return fail_internal("work exceeds a workspace list or scratch area");
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
                                          B.keys1, B.hdl0, B.hdl1, B.pos64, B.text, B.srank, B.cmap, b.bwt, B.start_row);
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
    if (nbig > Lo.cap_big) return fail_internal("work exceeds a workspace list or scratch area");
    g_stats.levels++;
    g_stats.host_levels++;
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
        T.begin();
        if ((rc = launch_local(B, b.tu, nb, b.rmax, b.bwt, (uint32_t)Lo.cap_chunks, counters + C_NCHUNK, st,
                               grid_from(seen(lv).nchunks, 0))))
          return rc;
        T.end(PH_LOCAL);
        T.begin();
        if ((rc = finish_finals_dev(b, st, grid_from(seen(lv).ftiles, PG_EMIT)))) return rc;
        T.end(PH_FINAL);
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

// The stringword schedule (Section 3.2) over one collection: for every
// window from the last to the first, its keys in position order, permuted
// into the current order, then one stable pass per varying digit, least
// significant first; finally the rows and term_pos.
int run_stringword(const Build &b, PhaseTimer &T, hipStream_t st) {
  constexpr int TI = 8, NW = 4;
  constexpr uint32_t TL = 64 * NW * TI;
  const Buffers &B = b.B;
  const Layout &Lo = b.Lo;
  const uint64_t nb = b.nb;
  g_stats.schedule = CXBWT_SCHEDULE_STRINGWORD;
  if (b.ncoll) CX_CHECK(hipMemcpyAsync(B.cmap, b.cm.data(), sizeof(CollMap), hipMemcpyHostToDevice, st));
  if (nb) {
    const uint64_t ntiles = ceil_div(nb, TL), ngroups = ceil_div(ntiles, GROUP_TILES);
    if (ntiles > Lo.max_tiles || ngroups > Lo.max_groups || ntiles > 0x7FFFFFFFull) return fail_internal("work exceeds a workspace list or scratch area");
    const uint32_t tp[2] = {0, (uint32_t)ntiles}, gp[2] = {0, (uint32_t)ngroups};
    CX_CHECK(hipMemcpyAsync(B.tile_prefix, tp, sizeof(tp), hipMemcpyHostToDevice, st));
    CX_CHECK(hipMemcpyAsync(B.group_prefix, gp, sizeof(gp), hipMemcpyHostToDevice, st));
    uint64_t *K[2] = {B.keys0, B.keys1};
    uint32_t *H[2] = {B.hdl0, B.hdl1};
    unsigned long long *orand = B.seg_or;  // OR and AND of a window's ordering bits
    const unsigned grid = (unsigned)std::min<uint64_t>(ceil_div(nb, BLOCK), 65536);
    int cur = 0, rc;
    for (int w = (int)b.rmax - 1; w >= 0; --w) {
      if ((rc = fill_u64((uint64_t *)orand, 1, 0, st))) return rc;
      if ((rc = fill_u64((uint64_t *)orand + 1, 1, ~0ull, st))) return rc;
      T.begin();
      k_sched_window<<<grid, BLOCK, 0, st>>>(B.text, B.srank, nb, (uint32_t)w, K[1 - cur], orand);
      CX_LAUNCHED();
      k_sched_gather<<<grid, BLOCK, 0, st>>>(K[1 - cur], nb, w == (int)b.rmax - 1, K[cur], H[cur]);
      CX_LAUNCHED();
      T.end(PH_GEN);
      uint64_t oa[2];
      CX_CHECK(hipMemcpyAsync(oa, orand, sizeof(oa), hipMemcpyDeviceToHost, st));
      CX_CHECK(hipStreamSynchronize(st));
      T.collect();
      g_stats.window_fetches += nb;
      for (int d = 7; d >= 0; --d) {
        if (((oa[0] ^ oa[1]) & digit_mask(d)) == 0) continue;  // constant digit: the pass would not move anything
        T.begin();
        k_sched_hist<TL><<<(unsigned)ntiles, BLOCK, 0, st>>>(K[cur], nb, d, B.tile_hist);
        CX_LAUNCHED();
        T.end(PH_HIST);
        T.begin();
        k_group_scan<false><<<(unsigned)ngroups, BLOCK, 0, st>>>(B.tile_prefix, B.group_prefix, 1, nullptr,
                                                                 B.tile_hist, B.gsum);
        CX_LAUNCHED();
        k_sched_top<<<1, 64, 0, st>>>(B.gsum, (uint32_t)ngroups);
        CX_LAUNCHED();
        T.end(PH_SCAN);
        T.begin();
        k_sched_scatter<TI, NW><<<(unsigned)ntiles, 64 * NW, 0, st>>>(K[cur], H[cur], nb, d, B.tile_hist, B.gsum,
                                                                      K[1 - cur], H[1 - cur]);
        CX_LAUNCHED();
        T.end(PH_SCATTER);
        cur = 1 - cur;
        g_stats.levels++;
        g_stats.scattered_suffixes += nb;
        g_stats.level_suffixes += nb;
      }
      g_stats.max_window = std::max<uint32_t>(g_stats.max_window, (uint32_t)w);
    }
    T.begin();
    k_sched_emit<<<grid, BLOCK, 0, st>>>(K[cur], H[cur], nb, B.cmap, B.text, B.srank, b.bwt, B.start_row);
    CX_LAUNCHED();
    T.end(PH_FINAL);
  }
  T.begin();
  k_term<<<grid_for(b.n, 256), 256, 0, st>>>(b.offsets, b.n, b.nb, B.text, B.srank, B.start_row, b.term_pos);
  CX_LAUNCHED();
  T.end(PH_FINAL);
  return CXBWT_OK;
}

// After a run of levels the device scheduled (a graph replay): the status,
// the statistics the device counted, and the levels it left to the host.
// hc0 holds the counters read after the run.
int finish_device_levels(const Build &b, const uint32_t (&hc0)[C_COUNT], PhaseTimer &T, hipStream_t st) {
  uint32_t hc[C_COUNT];
  memcpy(hc, hc0, sizeof(hc));
  int rc;
  if (hc[C_STATUS] & (ST_BAD_OFFSETS | ST_TOO_LONG)) return fail_status(hc[C_STATUS]);
  if (hc[C_STATUS]) return fail_status(hc[C_STATUS]);
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
  // the statistics block still holds the device levels' counts: take the rest only
  g_stats.window_fetches = 0;
  g_stats.scattered_suffixes = 0;
  if ((rc = read_totals(b, T, st, hc))) return rc;
  if (hc[C_STATUS]) return fail_status(hc[C_STATUS]);
  return CXBWT_OK;
}

// The whole build for ncoll collections laid end to end (a single build is
// one collection).  coll_reads (host) holds ncoll + 1 read boundaries.
int run_build(const uint64_t *packed, const uint64_t *offsets, uint64_t n, uint64_t nb, uint32_t maxlen,
              const uint64_t *coll_reads, uint32_t ncoll, uint8_t *bwt, uint64_t *term_pos, unsigned char *ws,
              hipStream_t st, bool allow_timing = true) {
  g_stats = cxbwt_stats{};
  g_last_error[0] = 0;
  PhaseTimer T{st, allow_timing && g_timing != 0, {}};
  Build b;
  build_init(b, packed, offsets, n, nb, maxlen, coll_reads, ncoll, bwt, term_pos, ws);
  int rc;
  if ((rc = enqueue_prep(b, b.coll_reads.data(), nullptr, T, st))) return rc;
  if ((rc = enqueue_records(b, T, st))) return rc;
  if ((rc = plan_level1(b, T, st))) return rc;
  if (ncoll == 1 && b.tu.schedule == CXBWT_SCHEDULE_STRINGWORD) {
    if ((rc = run_stringword(b, T, st))) return rc;
  } else {
    Level1Vectors v;
    v.make(b);
    level1_stats(b);
    if ((rc = enqueue_body(b, v.src, 0, T, st))) return rc;
  }
  uint32_t hc[C_COUNT];
  if ((rc = read_totals(b, T, st, hc))) return rc;
  if (hc[C_STATUS]) return fail_status(hc[C_STATUS]);
  return CXBWT_OK;
}

// ---- the build in ranges of window-0 key prefixes -------------------------

// A class of suffixes whose window-0 keys share their top `depth` digits
// (`prefix`, ordering bits only), and its size.
struct PrefixClass {
  uint64_t prefix;
  uint32_t depth;
  uint64_t count;
};
// A range: consecutive classes, keys lo..hi (ordering bits, inclusive), the
// rows after `before` suffixes of earlier ranges; its keys agree on their
// first `common` digits.
struct Range {
  uint64_t lo, hi, count, before;
  uint32_t common;
  uint64_t skip = 0;  // a piece of one class of identical suffixes: its first member in read order
};

// Ordering bits of the smallest and largest key with this prefix.
uint64_t class_lo(const PrefixClass &c) { return c.prefix; }
uint64_t class_hi(const PrefixClass &c) {
  if (c.depth >= 8) return c.prefix;
  if (c.depth == 0) return ~7ull;
  return (c.prefix | ((1ull << (64 - 8 * c.depth)) - 1)) & ~7ull;
}

// Counts the next digit of every class in `parents` (all of one depth, at
// most PH_MAX_PREFIXES, ascending) on the device; returns the child classes.
int count_children(const Build &b, const std::vector<PrefixClass> &parents, std::vector<PrefixClass> &children,
                   hipStream_t st) {
  const Buffers &B = b.B;
  const uint32_t np = (uint32_t)parents.size();
  const uint32_t depth = parents[0].depth;
  std::vector<uint64_t> pf(np);
  for (uint32_t i = 0; i < np; ++i) pf[i] = parents[i].prefix;
  std::vector<unsigned long long> cnt((size_t)np * 256);
  int rc;
  if ((rc = fill_u64((uint64_t *)B.ph_counts, (uint64_t)np * 256, 0, st))) return rc;
  CX_CHECK(hipMemcpyAsync(B.ph_prefixes, pf.data(), 8 * np, hipMemcpyHostToDevice, st));
  const uint64_t nrec = ceil_div(b.nb, 16);
  const unsigned grid = (unsigned)std::min<uint64_t>(ceil_div(nrec, BLOCK), 2048);
  const size_t lds = (size_t)np * 256 * 4 + (size_t)np * 8;
  k_prefix_hist<<<grid, BLOCK, lds, st>>>(B.text, b.nb, B.ph_prefixes, np, depth, B.ph_counts);
  CX_LAUNCHED();
  CX_CHECK(hipMemcpyAsync(cnt.data(), B.ph_counts, 8 * cnt.size(), hipMemcpyDeviceToHost, st));
  CX_CHECK(hipStreamSynchronize(st));
  const uint32_t nd = depth == 7 ? 32u : 256u;  // digit 7 is the 5-bit clamped length
  for (uint32_t i = 0; i < np; ++i)
    for (uint32_t v = 0; v < nd; ++v) {
      const uint64_t c = cnt[(size_t)i * 256 + v];
      if (!c) continue;
      const uint64_t bits = depth < 7 ? (uint64_t)v << (56 - 8 * depth) : (uint64_t)v << 3;
      children.push_back(PrefixClass{parents[i].prefix | bits, depth + 1, c});
    }
  return CXBWT_OK;
}

// Section 3.1's partitioning on the device: classes of window-0 key
// prefixes, refined one digit at a time while larger than m, packed in key
// order into ranges of at most m suffixes.  CXBWT_ERANGE when a class of
// identical window-0 keys alone exceeds m.
int plan_ranges(const Build &b, uint64_t m, std::vector<Range> &ranges, hipStream_t st) {
  std::vector<PrefixClass> leaves, todo{PrefixClass{0, 0, b.nb}};
  int rc;
  while (!todo.empty()) {
    // the shallowest classes first, up to PH_MAX_PREFIXES per counting pass
    std::sort(todo.begin(), todo.end(), [](const PrefixClass &x, const PrefixClass &y) {
      return x.depth != y.depth ? x.depth < y.depth : x.prefix < y.prefix;
    });
    size_t k = 1;
    while (k < todo.size() && k < (size_t)PH_MAX_PREFIXES && todo[k].depth == todo[0].depth) ++k;
    const std::vector<PrefixClass> parents(todo.begin(), todo.begin() + k);
    todo.erase(todo.begin(), todo.begin() + k);
    std::vector<PrefixClass> kids;
    if ((rc = count_children(b, parents, kids, st))) return rc;
    for (const PrefixClass &c : kids) {
      if (c.count <= m) leaves.push_back(c);
      else if (c.depth < 8) todo.push_back(c);
      else if (clamp_of(c.prefix) < (uint32_t)W) leaves.push_back(c);  // identical suffixes: cut by read order below
      else return CXBWT_ERANGE;  // equal whole first windows whose order depends on later windows
    }
  }
  std::sort(leaves.begin(), leaves.end(),
            [](const PrefixClass &x, const PrefixClass &y) { return x.prefix < y.prefix; });
  ranges.clear();
  uint64_t before = 0;
  bool open = false;  // the last range takes more classes
  for (const PrefixClass &c : leaves) {
    if (c.count > m) {
      // a class of identical suffixes (one whole first-window key that ends
      // inside the window) above the budget: their order is the read order,
      // so it is cut into pieces of m in that order, each a range of its own
      for (uint64_t k = 0; k < c.count; k += m) {
        Range r{c.prefix, c.prefix, std::min<uint64_t>(m, c.count - k), before, 0};
        r.skip = k;
        ranges.push_back(r);
        before += r.count;
      }
      open = false;
      continue;
    }
    if (!open || ranges.back().count + c.count > m) {
      ranges.push_back(Range{class_lo(c), class_hi(c), 0, before, 0});
      open = true;
    }
    Range &r = ranges.back();
    r.hi = class_hi(c);
    r.count += c.count;
    before += c.count;
  }
  for (Range &r : ranges) {
    uint32_t j = 0;
    while (j < 8 && digit_of(r.lo, (int)j) == digit_of(r.hi, (int)j)) ++j;
    r.common = j;
  }
  return CXBWT_OK;
}

// Lists the suffixes of range `r` into keys0 / hdl0 [0, count), in position
// order.
int list_range(const Build &b, const Range &r, PhaseTimer &T, hipStream_t st) {
  const Buffers &B = b.B;
  const Layout &Lo = b.Lo;
  const uint64_t ntl = ceil_div(b.nb, LIST_TILE);
  const uint64_t nlb = ceil_div(ntl, RANK_BLOCK_WORDS);
  if (ntl + 1 > Lo.n_list_tiles || nlb + 1 > Lo.n_list_blocks || r.count > Lo.sort_cap) return fail_internal("work exceeds a workspace list or scratch area");
  T.begin();
  k_range_count<<<(unsigned)ntl, BLOCK, 0, st>>>(B.text, b.nb, r.lo, r.hi, B.list_tiles);
  CX_LAUNCHED();
  k_count_blocks<<<(unsigned)nlb, BLOCK, 0, st>>>(B.list_tiles, ntl, B.list_blocks);
  CX_LAUNCHED();
  k_rank_top<<<1, BLOCK, 0, st>>>(B.list_blocks, (uint32_t)nlb);
  CX_LAUNCHED();
  k_count_prefix<<<(unsigned)nlb, BLOCK, 0, st>>>(B.list_tiles, ntl, B.list_blocks);
  CX_LAUNCHED();
  k_range_list<<<(unsigned)ntl, BLOCK, 0, st>>>(B.text, b.nb, r.lo, r.hi, B.list_tiles, r.skip, r.count, B.keys0,
                                                 B.hdl0, B.pos64);
  CX_LAUNCHED();
  T.end(PH_GEN);
  return CXBWT_OK;
}

// One collection built in ranges of at most m suffixes: the bare
// terminators and text records as for a whole build, the ranges planned
// from prefix counts, then each range listed, sorted (levels and chunks) and
// emitted at its rows; term_pos at the end.
int run_range_build(const uint64_t *packed, const uint64_t *offsets, uint64_t n, uint64_t nb, uint32_t maxlen,
                    uint64_t m, bool wide, uint8_t *bwt, uint64_t *term_pos, unsigned char *ws, hipStream_t st) {
  g_stats = cxbwt_stats{};
  g_last_error[0] = 0;
  PhaseTimer T{st, g_timing != 0, {}};
  Build b;
  const uint64_t one[2] = {0, n};
  build_init(b, packed, offsets, n, nb, maxlen, one, 1, bwt, term_pos, ws, m, wide);
  int rc;
  if ((rc = enqueue_prep(b, b.coll_reads.data(), nullptr, T, st))) return rc;
  if ((rc = enqueue_records(b, T, st))) return rc;
  {  // the offsets are checked on the device before anything is listed
    uint32_t hc[C_COUNT];
    CX_CHECK(hipMemcpyAsync(hc, b.B.counters, sizeof(hc), hipMemcpyDeviceToHost, st));
    CX_CHECK(hipStreamSynchronize(st));
    T.collect();
    if (hc[C_STATUS] & (ST_BAD_OFFSETS | ST_TOO_LONG)) return fail_status(hc[C_STATUS]);
  }
  g_stats.chunk_suffixes = nb;
  std::vector<Range> ranges;
  if (nb) {
    if ((rc = plan_ranges(b, m, ranges, st))) return rc;
  }
  g_stats.ranges = (uint32_t)ranges.size();
  // every range's rows follow the n bare-terminator rows and the earlier ranges
  std::vector<CollMap> cm(ranges.size());
  std::vector<Seg> seg(ranges.size());
  for (size_t i = 0; i < ranges.size(); ++i) {
    cm[i].out_shift = n + ranges[i].before;
    cm[i].row_shift = (int64_t)(n + ranges[i].before);
  }
  for (size_t i = 0; i < ranges.size(); ++i) {
    const Range &r = ranges[i];
    // the row map of this range, in the one collection slot (stream order:
    // after the previous range's kernels have read theirs)
    CX_CHECK(hipMemcpyAsync(b.B.cmap, &cm[i], sizeof(CollMap), hipMemcpyHostToDevice, st));
    if ((rc = list_range(b, r, T, st))) return rc;
    const bool small = r.count <= (uint64_t)b.tu.chunk();
    // a range that fits a chunk: one unsplit chunk; else one segment whose
    // keys agree on their first `common` digits
    seg[i] = Seg{0, (uint32_t)r.count, 0, (uint8_t)std::min<uint32_t>(r.common, small ? 6 : 7), 0, 0,
                 (uint8_t)(small ? 1 : 0), 0};
    if (small) {
      CX_CHECK(hipMemcpyAsync(b.B.chunks, &seg[i], sizeof(Seg), hipMemcpyHostToDevice, st));
      if ((rc = finish_level(b.B, b.Lo, b.tu, nb, b.rmax, bwt, 1, 0, 0, 0, T, st))) return rc;
      continue;
    }
    CX_CHECK(hipMemcpyAsync(b.B.big_next, &seg[i], sizeof(Seg), hipMemcpyHostToDevice, st));
    LevelOut acc{};
    acc.next_len = r.count;
    acc.next_tiles = ceil_div(r.count, b.tile_len);
    acc.next_groups = ceil_div(acc.next_tiles, GROUP_TILES);
    if ((rc = run_levels(b, acc, 1, T, st))) return rc;
  }
  T.begin();
  k_term<<<grid_for(n, 256), 256, 0, st>>>(offsets, n, nb, b.B.text, b.B.srank, b.B.start_row, term_pos);
  CX_LAUNCHED();
  T.end(PH_FINAL);
  uint32_t hc[C_COUNT];
  if ((rc = read_totals(b, T, st, hc))) return rc;
  if (hc[C_STATUS]) return fail_status(hc[C_STATUS]);
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
  if (hc[C_STATUS]) return fail_status(hc[C_STATUS]);
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
  if (ec != hipSuccess || !g) return fail_hip(ec, "graph capture");
  P.graph = g;
  CX_CHECK(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
  return CXBWT_OK;
}

// After a replay: status, statistics, and the levels left to the host.
int graph_finish(GraphPlan &P, hipStream_t st) {
  PhaseTimer T{st, false, {}};
  g_stats = P.base;
  uint32_t hc[C_COUNT];
  int rc;
  if ((rc = read_totals(P.b, T, st, hc))) return rc;
  return finish_device_levels(P.b, hc, T, st);
}

}  // namespace

struct cxbwt_graph {
  GraphPlan p;
};

// A build started by cxbwt_build_start / cxbwt_build_batch_start: a worker
// thread enqueues it on the caller's stream and waits on that stream between
// levels; the caller waits for the job instead of for the call.
struct cxbwt_job {
  std::thread worker;
  std::atomic<int> done{0};
  int status = CXBWT_OK;
  cxbwt_stats stats{};
  char error[256] = "";
};

namespace {

struct JobArgs {
  const uint64_t *packed, *offsets;
  uint64_t n, nb;
  uint32_t maxlen;
  std::vector<uint64_t> coll_reads;  // copied at the call: the caller's array may go away
  uint8_t *bwt;
  uint64_t *term_pos;
  unsigned char *ws;
  hipStream_t st;
  int device;
  Tuning tu;   // the calling thread's choices at the call
  int timing;
};

void job_main(cxbwt_job *job, JobArgs a) {
  int rc = CXBWT_OK;
  try {
    if (hipSetDevice(a.device) != hipSuccess) {
      rc = CXBWT_EDEVICE;
    } else {
      g_tuning = a.tu;
      g_timing = a.timing;
      rc = run_build(a.packed, a.offsets, a.n, a.nb, a.maxlen, a.coll_reads.data(),
                     (uint32_t)(a.coll_reads.size() - 1), a.bwt, a.term_pos, a.ws, a.st);
      // a failed build may leave work in flight: the job ends when the stream has drained
      if (rc && hipStreamSynchronize(a.st) != hipSuccess) rc = CXBWT_EDEVICE;
    }
  } catch (...) {
    rc = CXBWT_EDEVICE;
    (void)hipStreamSynchronize(a.st);
  }
  job->stats = g_stats;
  job->status = rc;
  memcpy(job->error, g_last_error, sizeof(job->error));
  job->done.store(1, std::memory_order_release);
}

// The choices a started build runs with: opts, or the calling thread's.
bool job_choices(const cxbwt_opts *opts, Tuning &tu, int &timing) {
  if (!opts) {
    tu = g_tuning;
    timing = g_timing;
    return true;
  }
  if (!tuning_ok(opts->tile_items, opts->chunk_items)) return false;
  if (opts->schedule != CXBWT_SCHEDULE_MSD && opts->schedule != CXBWT_SCHEDULE_STRINGWORD) return false;
  tu.tile_items = opts->tile_items;
  tu.chunk_items = opts->chunk_items;
  tu.schedule = opts->schedule;
  timing = opts->timing ? 1 : 0;
  return true;
}

// A blocking build's choices: set for the call, the thread's restored after.
struct ChoiceScope {
  Tuning saved_tu;
  int saved_timing;
  ChoiceScope(const Tuning &tu, int timing) : saved_tu(g_tuning), saved_timing(g_timing) {
    g_tuning = tu;
    g_timing = timing;
  }
  ~ChoiceScope() {
    g_tuning = saved_tu;
    g_timing = saved_timing;
  }
};

int start_job(JobArgs &&a, cxbwt_job **out) {
  if (hipGetDevice(&a.device) != hipSuccess) return CXBWT_EDEVICE;
  cxbwt_job *job = new (std::nothrow) cxbwt_job;
  if (!job) return CXBWT_ENOMEM;
  try {
    job->worker = std::thread(job_main, job, std::move(a));
  } catch (...) {
    delete job;
    return CXBWT_EDEVICE;
  }
  *out = job;
  return CXBWT_OK;
}

}  // namespace

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
    if (((uintptr_t)p & 255u) != 0) return fail_internal("work exceeds a workspace list or scratch area");
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
  if (n_bases > CXBWT_MAX_RANGE_BASES) return CXBWT_ERANGE;
  if (!packed || (n_bases && !ascii)) return CXBWT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (d_status) {
    int rc = fill_u32(d_status, 1, 0, st);
    if (rc) return rc;
  }
  const uint64_t nw = cxbwt_packed_words(n_bases);
  k_pack<<<grid_for(nw, 256), 256, 0, st>>>(ascii, n_bases, packed, nw, d_status);
  CX_LAUNCHED();
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
                const cxbwt_opts *opts, void *stream) {
  if (!packed || !offsets || !bwt || !term_pos || !workspace || n_reads == 0) return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (workspace_bytes < cxbwt_workspace_bytes(n_reads, n_bases, max_read_len)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  Tuning tu;
  int timing = 0;
  if (!job_choices(opts, tu, timing)) return CXBWT_EINVAL;
  ChoiceScope scope(tu, timing);
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

size_t cxbwt_range_workspace_bytes(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len,
                                   uint64_t max_range_suffixes, uint32_t flags) {
  if (!range_sizes_ok(n_reads, n_bases, max_read_len, max_range_suffixes, flags)) return 0;
  return (size_t)make_layout(n_reads, n_bases, 1, max_range_suffixes, range_wide(n_bases, flags)).total;
}

int cxbwt_build_ranges(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                       uint32_t max_read_len, uint64_t max_range_suffixes, uint32_t flags, uint8_t *bwt,
                       uint64_t *term_pos, void *workspace, size_t workspace_bytes, void *stream) {
  if (!packed || !offsets || !bwt || !term_pos || !workspace || n_reads == 0 || max_range_suffixes == 0 ||
      (flags & ~(uint32_t)CXBWT_RANGE_WIDE))
    return CXBWT_EINVAL;
  if (!range_sizes_ok(n_reads, n_bases, max_read_len, max_range_suffixes, flags)) return CXBWT_ERANGE;
  if (workspace_bytes < cxbwt_range_workspace_bytes(n_reads, n_bases, max_read_len, max_range_suffixes, flags))
    return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  return run_range_build(packed, offsets, n_reads, n_bases, max_read_len, max_range_suffixes,
                         range_wide(n_bases, flags), bwt, term_pos, (unsigned char *)workspace, (hipStream_t)stream);
}

int cxbwt_build_start(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                      uint32_t max_read_len, uint8_t *bwt, uint64_t *term_pos, void *workspace,
                      size_t workspace_bytes, const cxbwt_opts *opts, void *stream, cxbwt_job **job) {
  if (!job) return CXBWT_EINVAL;
  *job = nullptr;
  if (!packed || !offsets || !bwt || !term_pos || !workspace || n_reads == 0) return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (workspace_bytes < cxbwt_workspace_bytes(n_reads, n_bases, max_read_len)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  JobArgs a{packed, offsets, n_reads, n_bases, max_read_len, {0, n_reads}, bwt, term_pos,
            (unsigned char *)workspace, (hipStream_t)stream, 0, Tuning{8, 6}, 0};
  if (!job_choices(opts, a.tu, a.timing)) return CXBWT_EINVAL;
  return start_job(std::move(a), job);
}

int cxbwt_build_batch_start(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                            uint32_t max_read_len, const uint64_t *coll_reads, uint32_t n_coll, uint8_t *bwt,
                            uint64_t *term_pos, void *workspace, size_t workspace_bytes,
                            const cxbwt_opts *opts, void *stream, cxbwt_job **job) {
  if (!job) return CXBWT_EINVAL;
  *job = nullptr;
  if (!packed || !offsets || !bwt || !term_pos || !workspace || !coll_reads || n_reads == 0 || n_coll == 0)
    return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (n_coll > n_reads) return CXBWT_EINVAL;
  if (coll_reads[0] != 0 || coll_reads[n_coll] != n_reads) return CXBWT_EINVAL;
  for (uint32_t c = 0; c < n_coll; ++c)
    if (coll_reads[c + 1] <= coll_reads[c]) return CXBWT_EINVAL;
  if (workspace_bytes < cxbwt_batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  JobArgs a{packed, offsets, n_reads, n_bases, max_read_len,
            std::vector<uint64_t>(coll_reads, coll_reads + n_coll + 1), bwt, term_pos,
            (unsigned char *)workspace, (hipStream_t)stream, 0, Tuning{8, 6}, 0};
  if (!job_choices(opts, a.tu, a.timing)) return CXBWT_EINVAL;
  return start_job(std::move(a), job);
}

int cxbwt_job_done(const cxbwt_job *job) { return job && job->done.load(std::memory_order_acquire) ? 1 : 0; }

int cxbwt_job_wait(cxbwt_job *job, cxbwt_stats *stats) {
  if (!job) return CXBWT_EINVAL;
  if (job->worker.joinable()) job->worker.join();
  const int rc = job->status;
  if (stats) *stats = job->stats;
  g_stats = job->stats;  // cxbwt_last_stats and cxbwt_last_error on the waiting thread
  memcpy(g_last_error, job->error, sizeof(g_last_error));
  delete job;
  return rc;
}

int cxbwt_build_batch(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                      uint32_t max_read_len, const uint64_t *coll_reads, uint32_t n_coll, uint8_t *bwt,
                      uint64_t *term_pos, void *workspace, size_t workspace_bytes, const cxbwt_opts *opts,
                      void *stream) {
  if (!packed || !offsets || !bwt || !term_pos || !workspace || !coll_reads || n_reads == 0 || n_coll == 0)
    return CXBWT_EINVAL;
  if (!sizes_ok(n_reads, n_bases, max_read_len)) return CXBWT_ERANGE;
  if (n_coll > n_reads) return CXBWT_EINVAL;
  if (coll_reads[0] != 0 || coll_reads[n_coll] != n_reads) return CXBWT_EINVAL;
  for (uint32_t c = 0; c < n_coll; ++c)
    if (coll_reads[c + 1] <= coll_reads[c]) return CXBWT_EINVAL;  // every collection holds a read
  if (workspace_bytes < cxbwt_batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll)) return CXBWT_ENOMEM;
  if (((uintptr_t)workspace & 255u) != 0) return CXBWT_EINVAL;
  Tuning tu;
  int timing = 0;
  if (!job_choices(opts, tu, timing)) return CXBWT_EINVAL;
  ChoiceScope scope(tu, timing);
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
  g_tuning.tile_items = tile_items;
  g_tuning.chunk_items = chunk_items;
  return CXBWT_OK;
}

int cxbwt_set_schedule(uint32_t schedule) {
  if (schedule != CXBWT_SCHEDULE_MSD && schedule != CXBWT_SCHEDULE_STRINGWORD) return CXBWT_EINVAL;
  g_tuning.schedule = schedule;
  return CXBWT_OK;
}

int cxbwt_get_schedule(uint32_t *schedule) {
  if (!schedule) return CXBWT_EINVAL;
  *schedule = g_tuning.schedule;
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

const char *cxbwt_last_error(void) { return g_last_error; }

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
