/*
 * cxbwt.h -- C ABI of the MI355X (gfx950) multi-string BWT library.
 *
 * The library builds the Burrows-Wheeler transform of a collection of reads
 * as defined in Section 2 of Liu, Luo & Lam, "GPU-Accelerated BWT
 * Construction for Large Collection of Short Reads" (the CX1 method):
 *
 *   * read r_i (bases A<C<G<T) is extended to S_i = r_i $_i;
 *   * the terminators sort below every base and $_i < $_j exactly when i < j;
 *   * all sum_i (L_i + 1) suffixes of all S_i are sorted lexicographically;
 *   * row rho of the BWT is the symbol before the rho-th suffix in its own
 *     string, or '$' when that suffix starts at offset 0 (Fig. 1 shows the
 *     collection {ACGT, TAGT, GGAA} giving TTAAG$TAG$CAGG$).
 *
 * Every step runs in HIP kernels on the device; the host code only checks
 * arguments, sizes the workspace and sequences launches.
 *
 * Conventions shared by all entry points
 *   * Pointers marked (device) must point to memory on the current HIP device;
 *     (host) pointers to host memory.  The caller allocates and frees every
 *     buffer, including the workspace; the library frees nothing it was
 *     given and keeps no device memory of its own apart from the fixed array
 *     behind cxbwt_build_noalloc.
 *   * `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   * Return value: one of the CXBWT_* status codes below.  No C++ exception
 *     crosses this interface.  cxbwt_status_str() gives a message.
 *   * Calls on distinct streams with distinct workspaces may run concurrently
 *     from different host threads.
 */
#ifndef CXBWT_H
#define CXBWT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define CXBWT_OK 0
#define CXBWT_EINVAL (-1)  /* a null pointer or inconsistent sizes            */
#define CXBWT_ERANGE (-2)  /* a size the library does not support (below)     */
#define CXBWT_ENOMEM (-3)  /* workspace smaller than cxbwt_workspace_bytes()  */
#define CXBWT_EDEVICE (-4) /* a HIP launch or runtime call failed             */
#define CXBWT_EDATA (-5)   /* the device found invalid input data: offsets not
                              a non-decreasing partition of the bases, a read
                              longer than max_read_len, or a non-ACGT byte     */
#define CXBWT_ESCRATCH (-6) /* cxbwt_build_noalloc: the input needs more
                               workspace than CXBWT_NOALLOC_WORKSPACE_BYTES   */

/* Largest supported n_bases: suffix handles are 32-bit base positions. */
#define CXBWT_MAX_BASES 4294967295ull
/* Largest n_bases of cxbwt_build_ranges (and cxbwt_pack): positions kept in
 * 64 bits per listed suffix, with 32-bit handles inside one range. */
#define CXBWT_MAX_RANGE_BASES (1ull << 38)
/* Largest supported max_read_len. */
#define CXBWT_MAX_READ_LEN 65535u

/*
 * The choices of one build (cxbwt_build, cxbwt_build_batch and the builds
 * that return at once): the kernel instantiation, the sort schedule and
 * per-class kernel timing, as cxbwt_set_tuning, cxbwt_set_schedule and
 * cxbwt_set_timing would set them, and checked the same way (CXBWT_EINVAL
 * for values those calls refuse).  A NULL opts takes the calling thread's
 * choices.  The result of a build never depends on them, only its speed.
 */
typedef struct cxbwt_opts {
  uint32_t tile_items;   /* 6, 8 or 16, as cxbwt_set_tuning          */
  uint32_t chunk_items;  /* 3, 6 or 8, as cxbwt_set_tuning           */
  uint32_t schedule;     /* CXBWT_SCHEDULE_MSD or _STRINGWORD       */
  uint32_t timing;       /* nonzero: per-class kernel times in stats */
} cxbwt_opts;

/*
 * Packed read layout (input of cxbwt_build), fixed by this library:
 * base t of the reads concatenated in read order is the 2-bit code
 * A=0, C=1, G=2, T=3 stored in 64-bit word t/32 at bits
 * [62 - 2*(t%32), 63 - 2*(t%32)], i.e. the first base of a word in its two
 * most significant bits.  A packed array holds cxbwt_packed_words(n_bases)
 * words: ceil(n_bases/32) data words plus one zero pad word.
 */
uint64_t cxbwt_packed_words(uint64_t n_bases);

/*
 * cxbwt_pack -- read packing (the 2-bit representation of Section 3, used
 * there to size the explicit-suffix alternative; here the device input form).
 * Up to CXBWT_MAX_RANGE_BASES bases.
 *
 *   ascii     (device) n_bases bytes, each 'A', 'C', 'G' or 'T'.
 *   n_bases   number of bases.
 *   packed    (device, out) cxbwt_packed_words(n_bases) uint64 words in the
 *             layout above; the pad word is written as zero.
 *   d_status  (device, out, may be NULL) one uint32 set to 0 and then to a
 *             non-zero value if any byte is not A/C/G/T (such bytes pack as
 *             A).  Read it after the stream completes.
 *   stream    hipStream_t as void*.
 * Asynchronous on `stream`.  Returns CXBWT_EINVAL for null ascii/packed with
 * n_bases > 0, CXBWT_ERANGE above CXBWT_MAX_RANGE_BASES, CXBWT_EDEVICE on a launch
 * failure.
 */
int cxbwt_pack(const uint8_t *ascii, uint64_t n_bases, uint64_t *packed, uint32_t *d_status,
               void *stream);

/*
 * cxbwt_workspace_bytes -- device workspace cxbwt_build needs for these
 * sizes (about 28 bytes per base plus small lists).  Pure host arithmetic:
 * no device call, usable without a GPU.  Returns 0 when the sizes are out of
 * range (see cxbwt_build).
 */
size_t cxbwt_workspace_bytes(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len);

/*
 * cxbwt_build -- the multi-string BWT of one read collection (Section 2;
 * the suffix sort of Section 3.2 done entirely on the device).
 *
 * Inputs
 *   packed        (device) cxbwt_packed_words(n_bases) words, layout above.
 *   offsets       (device) n_reads + 1 uint64: read i is bases
 *                 [offsets[i], offsets[i+1]) of the concatenation; offsets[0]
 *                 must be 0, offsets must not decrease, offsets[n_reads] must
 *                 equal n_bases.  Empty reads (equal neighbours) are allowed.
 *   n_reads       number of reads n (>= 1, < 2^32).
 *   n_bases       total bases B (<= CXBWT_MAX_BASES).
 *   max_read_len  an upper bound on every read length (<= CXBWT_MAX_READ_LEN);
 *                 it bounds the number of refinement windows.
 * Outputs
 *   bwt           (device, out) n_bases + n_reads bytes, ASCII over A/C/G/T/$:
 *                 row rho is the symbol before the rho-th smallest suffix.
 *   term_pos      (device, out) n_reads uint64: term_pos[i] is the row of the
 *                 offset-0 suffix of read i, i.e. the '$' row standing for
 *                 read i.  The '$' rows are exactly the values of term_pos.
 * Workspace
 *   workspace     (device) at least cxbwt_workspace_bytes(...) bytes, aligned
 *                 to 256 bytes; contents on entry are ignored.
 * Options
 *   opts          (host, may be NULL) this build's choices (cxbwt_opts); NULL
 *                 takes the calling thread's.  The thread's choices are left
 *                 as they were.
 * Behaviour
 *   Work is enqueued on `stream`; the call reads a few counters back between
 *   sort levels, so it returns only after the device work is complete.
 *   Returns CXBWT_EINVAL (null pointer, n_reads == 0), CXBWT_ERANGE (sizes
 *   above the limits), CXBWT_ENOMEM (workspace too small), CXBWT_EDATA
 *   (offsets invalid or a read longer than max_read_len, found on the device
 *   before any sorting; outputs are then unspecified), CXBWT_EDEVICE.
 */
int cxbwt_build(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                uint32_t max_read_len, uint8_t *bwt, uint64_t *term_pos, void *workspace,
                size_t workspace_bytes, const cxbwt_opts *opts, void *stream);

/*
 * cxbwt_build_noalloc -- cxbwt_build without a caller workspace and without
 * any device allocation, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc).  It waits on the
 * stream between sort levels as cxbwt_build does, so it is not a call to
 * make under HIP graph capture.
 *
 * The workspace is a fixed array of CXBWT_NOALLOC_WORKSPACE_BYTES in the
 * library's device code object: each device the library runs on holds its
 * own copy from the library's first use on it until the process ends.  The
 * call still takes the caller's inputs and outputs (packed, offsets, bwt,
 * term_pos: device pointers, meanings, layouts and data checks as for
 * cxbwt_build).  The first call on a device looks up that device's copy
 * (hipGetSymbolAddress) with the device current; no call allocates or frees
 * device memory, and kernel timing (cxbwt_set_timing) is not applied.
 *
 * Every call on one device shares that device's array and leaves its last
 * contents there; the build clears what it needs cleared itself.  Calls that
 * overlap on one device (two host threads, or two streams whose work is not
 * ordered) race on the array and give unspecified outputs.
 *
 * Returns as cxbwt_build, and CXBWT_ESCRATCH (before any HIP call) when
 * cxbwt_workspace_bytes(n_reads, n_bases, max_read_len) exceeds
 * CXBWT_NOALLOC_WORKSPACE_BYTES (about 9.7 Mbases of 100-base reads).
 */
#define CXBWT_NOALLOC_WORKSPACE_BYTES (256ull << 20)
int cxbwt_build_noalloc(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                        uint32_t max_read_len, uint8_t *bwt, uint64_t *term_pos, void *stream);

/*
 * The build in ranges -- Section 3.1's partitioning of the suffixes by their
 * leading characters (Fig. 2 steps 1-3): the suffixes are counted by the
 * top digits of their first 27-base window key, prefix classes larger than
 * the budget are counted again one 8-bit digit deeper, and consecutive
 * classes are packed in key order into ranges of at most
 * max_range_suffixes suffixes.  Each range is listed from the text on its
 * own (one scan of every position per range), sorted and refined like a
 * whole collection, and written at the BWT rows after the ranges below it;
 * the concatenation is the BWT.  The sort buffers hold one range at a time,
 * so the workspace is about 1.3 bytes per base for the text plus 27.5 bytes
 * per suffix of the largest range (cxbwt_range_workspace_bytes), against
 * 27.5 bytes per base for cxbwt_build.
 *
 * Collections above CXBWT_MAX_BASES bases (up to CXBWT_MAX_RANGE_BASES) are
 * built this way only: the suffixes of a range are then named by 32-bit
 * indices into a table of their 64-bit base positions (8 more bytes per
 * suffix of a range, one more load per later-window fetch), the indirection
 * Section 3.2 describes for sorting by index.  CXBWT_RANGE_WIDE asks for
 * that form below the limit too.
 *
 * cxbwt_range_workspace_bytes -- workspace for these sizes, budget and
 *   flags; pure host arithmetic, 0 when out of range.
 *
 * cxbwt_build_ranges -- arguments and results as cxbwt_build (one
 *   collection; the output is identical), plus
 *     max_range_suffixes  the most suffixes one range may hold
 *                         (1 .. CXBWT_MAX_BASES).
 *     flags               0 or CXBWT_RANGE_WIDE.
 *   n_bases may reach CXBWT_MAX_RANGE_BASES.  Returns as cxbwt_build,
 *   CXBWT_EINVAL for unknown flags, CXBWT_ENOMEM below
 *   cxbwt_range_workspace_bytes(), and CXBWT_ERANGE when more than
 *   max_range_suffixes suffixes share one whole first-window key (the
 *   partitioning cannot split them).  It waits on the stream between the
 *   counting passes, ranges and levels; cxbwt_last_stats().ranges gives the
 *   number of ranges.
 */
#define CXBWT_RANGE_WIDE 1u
size_t cxbwt_range_workspace_bytes(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len,
                                   uint64_t max_range_suffixes, uint32_t flags);
int cxbwt_build_ranges(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                       uint32_t max_read_len, uint64_t max_range_suffixes, uint32_t flags, uint8_t *bwt,
                       uint64_t *term_pos, void *workspace, size_t workspace_bytes, void *stream);

/*
 * cxbwt_batch_workspace_bytes -- workspace of cxbwt_build_batch for these
 * totals (same per-base cost as cxbwt_workspace_bytes plus per-collection
 * tables).  Pure host arithmetic; 0 when out of range or n_coll is 0 or
 * larger than n_reads.
 */
size_t cxbwt_batch_workspace_bytes(uint64_t n_reads, uint64_t n_bases, uint32_t max_read_len, uint32_t n_coll);

/*
 * cxbwt_build_batch -- the BWTs of n_coll independent collections in one
 * pass of the device pipeline: every sort level and every finishing launch
 * covers all collections at once (each collection is its own segment from
 * the first level on, so suffixes of different collections never meet).
 * Each result is exactly the cxbwt_build result of that collection alone
 * (Section 2 applied per collection).
 *
 * Inputs
 *   packed, offsets, n_reads, n_bases, max_read_len
 *                 the reads of all collections concatenated, collection
 *                 after collection, as for cxbwt_build (n_bases is the
 *                 total, at most CXBWT_MAX_BASES; offsets are global).
 *   coll_reads    (host) n_coll + 1 uint64: collection c holds reads
 *                 [coll_reads[c], coll_reads[c+1]); coll_reads[0] == 0,
 *                 strictly increasing (no empty collection), coll_reads[n_coll]
 *                 == n_reads.
 * Outputs
 *   bwt           (device, out) n_bases + n_reads bytes: the collections'
 *                 BWTs concatenated in order; collection c's BWT (n_c + B_c
 *                 bytes) starts at byte (reads before c) + (bases before c).
 *   term_pos      (device, out) n_reads uint64: for global read i of
 *                 collection c, the row inside collection c's BWT of the '$'
 *                 standing for read i - coll_reads[c].
 * Workspace, options, stream, return codes: as cxbwt_build, with CXBWT_EINVAL
 * also for inconsistent coll_reads and CXBWT_ENOMEM below
 * cxbwt_batch_workspace_bytes().  The stringword schedule applies to a
 * single collection only; a batch sorts most significant digit first.
 * Returns after the device work completes.
 */
int cxbwt_build_batch(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                      uint32_t max_read_len, const uint64_t *coll_reads, uint32_t n_coll, uint8_t *bwt,
                      uint64_t *term_pos, void *workspace, size_t workspace_bytes, const cxbwt_opts *opts,
                      void *stream);

/*
 * Builds that return at once (for callers that overlap builds with other
 * host work or with each other, such as a serving loop).
 *
 * cxbwt_build_start / cxbwt_build_batch_start -- arguments, checks and
 *   results as cxbwt_build / cxbwt_build_batch, plus
 *     job   (host, out) the started build, or NULL on an error returned here.
 *   Argument errors are returned by the call, before any HIP call; a started
 *   build's own status (CXBWT_EDATA and so on) comes from cxbwt_job_wait.  A
 *   library worker thread enqueues the build's kernels and copies on
 *   `stream`, in the order cxbwt_build would, and waits on that stream
 *   between sort levels (the level counts are read back); the calling thread
 *   does not wait.  Until cxbwt_job_wait returns, the caller keeps
 *   every buffer alive and unchanged and enqueues nothing on `stream` that
 *   reads the outputs.  Builds started on distinct streams with distinct
 *   workspaces run concurrently on the device; builds on one stream run one
 *   after the other.
 *
 * cxbwt_job_done -- 1 once the build's device work has completed (the
 *   outputs are final), else 0; never waits.  0 for NULL.
 *
 * cxbwt_job_wait -- wait for the build, return its status, copy its
 *   statistics to *stats (host, may be NULL; cxbwt_last_stats on the waiting
 *   thread also reads them) and free the job.  Every started job must be
 *   waited for exactly once.  CXBWT_EINVAL for NULL.
 */
typedef struct cxbwt_job cxbwt_job;
int cxbwt_build_start(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                      uint32_t max_read_len, uint8_t *bwt, uint64_t *term_pos, void *workspace,
                      size_t workspace_bytes, const cxbwt_opts *opts, void *stream, cxbwt_job **job);
int cxbwt_build_batch_start(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                            uint32_t max_read_len, const uint64_t *coll_reads, uint32_t n_coll, uint8_t *bwt,
                            uint64_t *term_pos, void *workspace, size_t workspace_bytes,
                            const cxbwt_opts *opts, void *stream, cxbwt_job **job);
int cxbwt_job_done(const cxbwt_job *job);
/* cxbwt_job_wait is declared after cxbwt_stats below. */

/*
 * A build captured once in a hipGraph and replayed (the batched row of the
 * design: every level's launches cover all collections, and the launches of
 * the levels after the first are sized on the device, so the whole build is
 * one graph with no host wait inside).  For callers that repeat builds of
 * one shape in fixed buffers: a serving loop, a pipeline stage.
 *
 * cxbwt_graph_create -- capture a build.  Arguments as cxbwt_build_batch
 *   (coll_reads may be NULL with n_coll == 1 for a single collection), plus
 *   levels        sort levels scheduled inside the graph, level 1 included;
 *                 0 = enough for any input of max_read_len (8 per 27-base
 *                 window, plus 2).  Each scheduled level that finds no work
 *                 costs a few empty launches.
 *   stream        the caller's stream: creation first runs one eager build
 *                 on it (it writes bwt and term_pos) and waits; the counts
 *                 each of its levels saw size the captured launches (larger
 *                 counts on a replay still run, looping).  The capture itself
 *                 uses a stream of its own.
 *   out           (host, out) the plan, or NULL on error.
 * The graph binds every pointer given here.  A replay is valid while the
 * buffers keep these sizes and every collection keeps its number of bases;
 * the read contents and the read lengths inside a collection may change.
 * Returns CXBWT_OK, CXBWT_EINVAL, CXBWT_ERANGE, CXBWT_ENOMEM, CXBWT_EDATA
 * (invalid offsets found by the eager pass) or CXBWT_EDEVICE.
 *
 * cxbwt_graph_launch -- enqueue one replay on `stream` and return at once.
 *
 * cxbwt_graph_finish -- wait for the replay on `stream`, check it and read
 *   its statistics (cxbwt_last_stats).  If the input needed more levels than
 *   were captured, or a level did not fit the per-segment scratch in one
 *   batch, the remaining levels run here on the host's schedule, with the
 *   same result.  Returns CXBWT_OK, CXBWT_EDATA (offsets or read lengths),
 *   CXBWT_EINVAL (the collection bases differ from the captured ones; the
 *   outputs are then unspecified) or CXBWT_EDEVICE.
 *
 * cxbwt_graph_destroy -- free the plan (NULL is ignored).  Calls that
 * overlap on one plan race; different plans need different workspaces.
 */
typedef struct cxbwt_graph cxbwt_graph;
int cxbwt_graph_create(const uint64_t *packed, const uint64_t *offsets, uint64_t n_reads, uint64_t n_bases,
                       uint32_t max_read_len, const uint64_t *coll_reads, uint32_t n_coll, uint8_t *bwt,
                       uint64_t *term_pos, void *workspace, size_t workspace_bytes, uint32_t levels, void *stream,
                       cxbwt_graph **out);
int cxbwt_graph_launch(cxbwt_graph *g, void *stream);
int cxbwt_graph_finish(cxbwt_graph *g, void *stream);
void cxbwt_graph_destroy(cxbwt_graph *g);

/* Counters describing the last cxbwt_build on the calling host thread. */
typedef struct cxbwt_stats {
  uint32_t levels;             /* global sort levels run                               */
  uint32_t max_window;         /* deepest 27-base key window used (0 = first window)   */
  uint64_t chunks;             /* bucket sets finished inside one wave                 */
  uint64_t big_segments;       /* segment passes run through the global levels         */
  uint64_t final_big;          /* groups of identical suffixes emitted from the levels */
  uint64_t chunk_suffixes;     /* suffixes finished inside waves                       */
  uint64_t level_suffixes;     /* suffix visits of the global histogram passes          */
  uint64_t scattered_suffixes; /* suffixes moved by global scatters                    */
  uint64_t regathered;         /* later-window keys fetched by the global levels        */
  uint64_t window_fetches;     /* later-window keys fetched inside waves                */
  /* regathered + window_fetches is the number of (suffix, window r >= 1)
   * pairs for which another suffix of the same collection shares the
   * suffix's first 27 r bases: only tied suffixes load a later window
   * (Section 3.2's stringword iterations, restricted to the ties).           */
  /* With timing on (cxbwt_set_timing): summed kernel time in ms and launch
   * count per kernel class: 0 prep, 1 key generation, 2 level histogram,
   * 3 level scan, 4 level scatter, 5 in-wave finish, 6 final emit.           */
  float ms[8];
  uint32_t launches[8];
  uint32_t level_batches;      /* batches the levels after the first ran in            */
  uint32_t ranges;             /* key ranges of a build in ranges (0 otherwise)        */
  uint32_t schedule;           /* CXBWT_SCHEDULE_* the build ran                       */
  uint32_t host_levels;        /* levels the host scheduled from counts it read back
                                * (0: the device scheduled every level)                 */
} cxbwt_stats;

/*
 * cxbwt_set_tuning -- pick, for later builds on the calling host thread, the
 * kernel instantiation the build uses (the library holds all of them):
 *   tile_items   suffixes per thread in a level tile of 256 threads (6 or 8),
 *                or 16: the wide tile of 4096 suffixes (512 threads x 8).
 *                Longer tiles write longer runs per bucket
 *   chunk_items  suffixes per lane of the one-wave chunk kernel (3, 6 or 8):
 *                the largest run of small buckets finished in LDS is 64 x this
 * The output is the same for every choice; only speed differs.  Default
 * (8, 6).  CXBWT_EINVAL for other values.  cxbwt_get_tuning reads the
 * current choice (CXBWT_EINVAL on NULL).  The workspace size does not depend
 * on the choice.  The autotuner in the Python package times the choices on a
 * sample of a workload and sets the fastest.
 */
int cxbwt_set_tuning(uint32_t tile_items, uint32_t chunk_items);
int cxbwt_get_tuning(uint32_t *tile_items, uint32_t *chunk_items);

/*
 * cxbwt_set_schedule -- the sort schedule of later single-collection builds
 * (cxbwt_build, cxbwt_build_noalloc) on the calling host thread:
 *   CXBWT_SCHEDULE_MSD         (default) most significant digit first on the
 *                              first 27-base window; later windows are
 *                              fetched for tied suffixes only, and small
 *                              buckets are finished in one wave.
 *   CXBWT_SCHEDULE_STRINGWORD  Section 3.2's schedule as the paper runs it:
 *                              a least-significant-digit radix sort of every
 *                              window of every suffix, last window first
 *                              (ceil((max_read_len + 1) / 27) windows, up to
 *                              eight 8-bit passes each, passes over a digit
 *                              no key varies in skipped), each window's keys
 *                              computed in base order and permuted into the
 *                              current order by handle (the paper's
 *                              "stringwords" permuted by index).
 * Both give the same output.  Batched builds and builds in ranges use the
 * MSD schedule.  CXBWT_EINVAL for another value; cxbwt_get_schedule reads it.
 */
#define CXBWT_SCHEDULE_MSD 0u
#define CXBWT_SCHEDULE_STRINGWORD 1u
int cxbwt_set_schedule(uint32_t schedule);
int cxbwt_get_schedule(uint32_t *schedule);

/* Copies the last build's counters (host) into *out; CXBWT_EINVAL on NULL. */
int cxbwt_last_stats(cxbwt_stats *out);

/* Waits for a started build (see cxbwt_build_start). */
int cxbwt_job_wait(cxbwt_job *job, cxbwt_stats *stats);

/*
 * cxbwt_set_timing -- for later cxbwt_build calls on the calling host thread,
 * bracket every kernel class with HIP events recorded on the build's stream
 * and sum their durations into cxbwt_stats.ms (enable != 0), or stop doing
 * so (enable == 0, the default).  Returns the previous setting.
 */
int cxbwt_set_timing(int enable);

/* Static message for a status code. */
const char *cxbwt_status_str(int status);

/*
 * cxbwt_last_error -- what lies behind the calling thread's last
 * CXBWT_EDEVICE or CXBWT_EDATA: the HIP error text of a failed runtime call
 * or launch, or the device's data checks that failed.  Empty after a build
 * that succeeded.  Valid until the thread's next build.
 */
const char *cxbwt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CXBWT_H */
