"""Thin Python binding of libcxbwt.so (argument marshalling only).

Every step of the BWT construction runs in the library's HIP kernels; this
module allocates device buffers with PyTorch, passes raw pointers and the
current stream through the C ABI declared in include/cxbwt.h, and turns status
codes into exceptions.  There is no CPU fallback: without the built library
every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcxbwt.so")

OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EDATA, ESCRATCH = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ERANGE: "ERANGE", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", EDATA: "EDATA",
                ESCRATCH: "ESCRATCH"}
# device array behind cxbwt_build_noalloc (CXBWT_NOALLOC_WORKSPACE_BYTES)
NOALLOC_WORKSPACE_BYTES = 256 << 20

# Names the C ABI exports (include/cxbwt.h).
ABI_FUNCTIONS = ("cxbwt_packed_words", "cxbwt_pack", "cxbwt_workspace_bytes", "cxbwt_build", "cxbwt_build_noalloc",
                 "cxbwt_range_workspace_bytes", "cxbwt_build_ranges", "cxbwt_batch_workspace_bytes", "cxbwt_build_batch",
                 "cxbwt_build_start", "cxbwt_build_batch_start", "cxbwt_job_done", "cxbwt_job_wait", "cxbwt_last_stats", "cxbwt_set_timing",
                 "cxbwt_set_tuning", "cxbwt_get_tuning", "cxbwt_set_schedule", "cxbwt_get_schedule", "cxbwt_graph_create", "cxbwt_graph_launch",
                 "cxbwt_graph_finish", "cxbwt_graph_destroy", "cxbwt_status_str", "cxbwt_last_error")

# kernel instantiations the library holds: (suffixes per thread in a level
# tile, suffixes per lane in a chunk); the first is the default
TUNING_CHOICES = ((8, 6), (8, 8), (8, 3), (6, 6), (6, 8), (6, 3), (16, 6), (16, 8), (16, 3))

# sort schedules (cxbwt_set_schedule): MSD with tie refinement (default), and
# Section 3.2's LSD passes over every window
SCHEDULE_MSD, SCHEDULE_STRINGWORD = 0, 1

# kernel classes of cxbwt_stats.ms / launches
KERNEL_CLASSES = ("prep", "gen", "level_hist", "level_scan", "level_scatter", "local", "final_emit", "unused")

_lock = threading.Lock()
_lib = None


class CxbwtError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str | None = None):
        self.status = status
        msg = lib().cxbwt_status_str(status).decode() if _lib is not None else ""
        if detail is None and _lib is not None and status in (EDEVICE, EDATA):
            detail = lib().cxbwt_last_error().decode()
        self.detail = detail or ""
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} ({msg})" +
                         (f": {self.detail}" if self.detail else ""))


class Opts(ctypes.Structure):
    """cxbwt_opts: the choices of one started build."""
    _fields_ = [("tile_items", ctypes.c_uint32), ("chunk_items", ctypes.c_uint32), ("schedule", ctypes.c_uint32),
                ("timing", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("max_window", ctypes.c_uint32), ("chunks", ctypes.c_uint64),
                ("big_segments", ctypes.c_uint64), ("final_big", ctypes.c_uint64),
                ("chunk_suffixes", ctypes.c_uint64), ("level_suffixes", ctypes.c_uint64),
                ("scattered_suffixes", ctypes.c_uint64), ("regathered", ctypes.c_uint64),
                ("window_fetches", ctypes.c_uint64), ("ms", ctypes.c_float * 8), ("launches", ctypes.c_uint32 * 8),
                ("level_batches", ctypes.c_uint32), ("ranges", ctypes.c_uint32), ("schedule", ctypes.c_uint32),
                ("host_levels", ctypes.c_uint32)]


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                                   "(python -m paper_1401_7457_amd.build)")
            L = ctypes.CDLL(LIB_PATH)
            vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
            L.cxbwt_packed_words.argtypes = [u64]
            L.cxbwt_packed_words.restype = u64
            L.cxbwt_pack.argtypes = [vp, u64, vp, vp, vp]
            L.cxbwt_pack.restype = ctypes.c_int
            L.cxbwt_workspace_bytes.argtypes = [u64, u64, u32]
            L.cxbwt_workspace_bytes.restype = ctypes.c_size_t
            L.cxbwt_build.argtypes = [vp, vp, u64, u64, u32, vp, vp, vp, ctypes.c_size_t, ctypes.POINTER(Opts), vp]
            L.cxbwt_build.restype = ctypes.c_int
            L.cxbwt_build_noalloc.argtypes = [vp, vp, u64, u64, u32, vp, vp, vp]
            L.cxbwt_build_noalloc.restype = ctypes.c_int
            L.cxbwt_range_workspace_bytes.argtypes = [u64, u64, u32, u64, u32]
            L.cxbwt_range_workspace_bytes.restype = ctypes.c_size_t
            L.cxbwt_build_ranges.argtypes = [vp, vp, u64, u64, u32, u64, u32, vp, vp, vp, ctypes.c_size_t, vp]
            L.cxbwt_build_ranges.restype = ctypes.c_int
            L.cxbwt_batch_workspace_bytes.argtypes = [u64, u64, u32, u32]
            L.cxbwt_batch_workspace_bytes.restype = ctypes.c_size_t
            L.cxbwt_build_batch.argtypes = [vp, vp, u64, u64, u32, vp, u32, vp, vp, vp, ctypes.c_size_t,
                                            ctypes.POINTER(Opts), vp]
            L.cxbwt_build_batch.restype = ctypes.c_int
            L.cxbwt_build_start.argtypes = [vp, vp, u64, u64, u32, vp, vp, vp, ctypes.c_size_t,
                                            ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
            L.cxbwt_build_start.restype = ctypes.c_int
            L.cxbwt_build_batch_start.argtypes = [vp, vp, u64, u64, u32, vp, u32, vp, vp, vp, ctypes.c_size_t,
                                                  ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
            L.cxbwt_build_batch_start.restype = ctypes.c_int
            L.cxbwt_job_done.argtypes = [vp]
            L.cxbwt_job_done.restype = ctypes.c_int
            L.cxbwt_job_wait.argtypes = [vp, ctypes.POINTER(Stats)]
            L.cxbwt_job_wait.restype = ctypes.c_int
            L.cxbwt_last_stats.argtypes = [ctypes.POINTER(Stats)]
            L.cxbwt_last_stats.restype = ctypes.c_int
            L.cxbwt_set_timing.argtypes = [ctypes.c_int]
            L.cxbwt_set_timing.restype = ctypes.c_int
            L.cxbwt_set_tuning.argtypes = [u32, u32]
            L.cxbwt_set_tuning.restype = ctypes.c_int
            L.cxbwt_get_tuning.argtypes = [ctypes.POINTER(u32), ctypes.POINTER(u32)]
            L.cxbwt_get_tuning.restype = ctypes.c_int
            L.cxbwt_set_schedule.argtypes = [u32]
            L.cxbwt_set_schedule.restype = ctypes.c_int
            L.cxbwt_get_schedule.argtypes = [ctypes.POINTER(u32)]
            L.cxbwt_get_schedule.restype = ctypes.c_int
            L.cxbwt_graph_create.argtypes = [vp, vp, u64, u64, u32, vp, u32, vp, vp, vp, ctypes.c_size_t, u32, vp,
                                             ctypes.POINTER(vp)]
            L.cxbwt_graph_create.restype = ctypes.c_int
            L.cxbwt_graph_launch.argtypes = [vp, vp]
            L.cxbwt_graph_launch.restype = ctypes.c_int
            L.cxbwt_graph_finish.argtypes = [vp, vp]
            L.cxbwt_graph_finish.restype = ctypes.c_int
            L.cxbwt_graph_destroy.argtypes = [vp]
            L.cxbwt_graph_destroy.restype = None
            L.cxbwt_status_str.argtypes = [ctypes.c_int]
            L.cxbwt_status_str.restype = ctypes.c_char_p
            L.cxbwt_last_error.argtypes = []
            L.cxbwt_last_error.restype = ctypes.c_char_p
            _lib = L
        return _lib


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def packed_words(n_bases: int) -> int:
    return int(lib().cxbwt_packed_words(n_bases))


def workspace_bytes(n_reads: int, n_bases: int, max_read_len: int) -> int:
    return int(lib().cxbwt_workspace_bytes(n_reads, n_bases, max_read_len))


def pack(ascii_dev, stream=None, out=None, status=None):
    """ASCII bases (uint8 CUDA tensor) -> packed words (int64 CUDA tensor holding uint64 bits)."""
    import torch
    if ascii_dev.dtype != torch.uint8 or not ascii_dev.is_cuda:
        raise TypeError("pack expects a uint8 CUDA tensor")
    ascii_dev = ascii_dev.contiguous()
    nb = ascii_dev.numel()
    if out is None:
        out = torch.empty(packed_words(nb), dtype=torch.int64, device=ascii_dev.device)
    elif out.numel() < packed_words(nb):
        raise ValueError("packed output too small")
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=ascii_dev.device)
    st = lib().cxbwt_pack(ctypes.c_void_p(ascii_dev.data_ptr() if nb else 0), nb, ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(status.data_ptr()), _stream_ptr(stream))
    if st != OK:
        raise CxbwtError(st, "cxbwt_pack")
    return out, status


def alloc_workspace(n_reads: int, n_bases: int, max_read_len: int, device="cuda"):
    import torch
    nbytes = workspace_bytes(n_reads, n_bases, max_read_len)
    if nbytes == 0:
        raise CxbwtError(ERANGE, "cxbwt_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def build(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, workspace=None, out=None, stream=None,
          opts=None):
    """BWT (uint8 CUDA tensor, n_bases + n_reads) and term_pos (int64 CUDA tensor, n_reads).

    packed: int64 CUDA tensor of packed words; offsets: int64 CUDA tensor of n_reads + 1 base offsets.
    opts: (tile_items, chunk_items, schedule[, timing]) for this build, else the thread's choices.
    """
    import torch
    dev = packed.device
    if workspace is None:
        workspace = alloc_workspace(n_reads, n_bases, max_read_len, dev)
    if out is None:
        bwt = torch.empty(n_bases + n_reads, dtype=torch.uint8, device=dev)
        term = torch.empty(n_reads, dtype=torch.int64, device=dev)
    else:
        bwt, term = out
    st = lib().cxbwt_build(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n_reads, n_bases,
                           max_read_len, ctypes.c_void_p(bwt.data_ptr()), ctypes.c_void_p(term.data_ptr()),
                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _opts(opts),
                           _stream_ptr(stream))
    if st != OK:
        raise CxbwtError(st, "cxbwt_build")
    return bwt, term


def build_noalloc(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, out, stream=None):
    """cxbwt_build_noalloc: the library's fixed device array is the workspace.

    out = (bwt, term) tensors the caller allocated (this call allocates no
    device memory).  Raises CxbwtError(ESCRATCH) when the input needs more
    than NOALLOC_WORKSPACE_BYTES of workspace.
    """
    bwt, term = out
    st = lib().cxbwt_build_noalloc(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n_reads,
                                   n_bases, max_read_len, ctypes.c_void_p(bwt.data_ptr()),
                                   ctypes.c_void_p(term.data_ptr()), _stream_ptr(stream))
    if st != OK:
        raise CxbwtError(st, "cxbwt_build_noalloc")
    return bwt, term


RANGE_WIDE = 1  # CXBWT_RANGE_WIDE: 64-bit positions in a table per range
MAX_BASES = (1 << 32) - 1  # CXBWT_MAX_BASES
MAX_RANGE_BASES = 1 << 38  # CXBWT_MAX_RANGE_BASES


def range_workspace_bytes(n_reads: int, n_bases: int, max_read_len: int, max_range_suffixes: int,
                          wide: bool = False) -> int:
    return int(lib().cxbwt_range_workspace_bytes(n_reads, n_bases, max_read_len, max_range_suffixes,
                                                 RANGE_WIDE if wide else 0))


def range_budget_for(n_reads: int, n_bases: int, max_read_len: int, workspace_bytes: int,
                     wide: bool = False) -> int:
    """Largest range budget (suffixes per range) whose workspace fits `workspace_bytes`,
    or 0 when even one suffix per range does not fit (host arithmetic only)."""
    def need(m):
        return range_workspace_bytes(n_reads, n_bases, max_read_len, m, wide)
    if need(1) == 0 or need(1) > workspace_bytes:
        return 0
    lo, hi = 1, max(1, min(n_bases, MAX_BASES))
    while lo < hi:  # the workspace grows with the budget
        mid = (lo + hi + 1) // 2
        if need(mid) <= workspace_bytes:
            lo = mid
        else:
            hi = mid - 1
    return lo


def build_ranges(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, max_range_suffixes: int,
                 workspace=None, out=None, stream=None, wide: bool = False):
    """cxbwt_build_ranges: the BWT built in ranges of at most max_range_suffixes suffixes
    (same result as `build`, a workspace sized by the largest range).  Collections above
    MAX_BASES bases use 64-bit positions by themselves; wide=True asks for them below it."""
    import torch
    dev = packed.device
    if workspace is None:
        nbytes = range_workspace_bytes(n_reads, n_bases, max_read_len, max_range_suffixes, wide)
        if nbytes == 0:
            raise CxbwtError(ERANGE, "cxbwt_range_workspace_bytes")
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if out is None:
        bwt = torch.empty(n_bases + n_reads, dtype=torch.uint8, device=dev)
        term = torch.empty(n_reads, dtype=torch.int64, device=dev)
    else:
        bwt, term = out
    st = lib().cxbwt_build_ranges(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n_reads,
                                  n_bases, max_read_len, int(max_range_suffixes), RANGE_WIDE if wide else 0,
                                  ctypes.c_void_p(bwt.data_ptr()),
                                  ctypes.c_void_p(term.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                                  workspace.numel(), _stream_ptr(stream))
    if st != OK:
        raise CxbwtError(st, "cxbwt_build_ranges")
    return bwt, term


def batch_workspace_bytes(n_reads: int, n_bases: int, max_read_len: int, n_coll: int) -> int:
    return int(lib().cxbwt_batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll))


def build_batch(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, coll_reads, workspace=None,
                out=None, stream=None, opts=None):
    """BWTs of several collections laid end to end (see cxbwt_build_batch).
    opts: as for build.

    coll_reads: host sequence of n_coll + 1 read boundaries.  Returns the
    concatenated BWTs (uint8 CUDA tensor) and per-read term_pos rows local to
    each collection (int64 CUDA tensor).
    """
    import torch
    cr = np.ascontiguousarray(np.asarray(coll_reads, dtype=np.uint64))
    n_coll = cr.size - 1
    dev = packed.device
    if workspace is None:
        nbytes = batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll)
        if nbytes == 0:
            raise CxbwtError(ERANGE, "cxbwt_batch_workspace_bytes")
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if out is None:
        bwt = torch.empty(n_bases + n_reads, dtype=torch.uint8, device=dev)
        term = torch.empty(n_reads, dtype=torch.int64, device=dev)
    else:
        bwt, term = out
    st = lib().cxbwt_build_batch(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n_reads,
                                 n_bases, max_read_len, cr.ctypes.data_as(ctypes.c_void_p), n_coll,
                                 ctypes.c_void_p(bwt.data_ptr()), ctypes.c_void_p(term.data_ptr()),
                                 ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _opts(opts),
                                 _stream_ptr(stream))
    if st != OK:
        raise CxbwtError(st, "cxbwt_build_batch")
    return bwt, term


class BuildJob:
    """A build started with build_start / build_batch_start (cxbwt_job).

    Holds every tensor the build reads or writes until wait() returns.
    done(): the device work has completed.  wait(): its status (raises on a
    failure) and (bwt, term).  A job must be waited for once.
    """

    def __init__(self, handle, what, tensors, out):
        self._h = handle
        self._what = what
        self._tensors = tensors
        self.bwt, self.term = out
        self.stats = None

    def done(self) -> bool:
        return bool(self._h) and bool(lib().cxbwt_job_done(self._h))

    def wait(self):
        if not self._h:
            raise RuntimeError("job already waited for")
        s = Stats()
        st = lib().cxbwt_job_wait(self._h, ctypes.byref(s))
        self._h = ctypes.c_void_p()
        self._tensors = None
        self.stats = _stats_dict(s)
        if st != OK:
            raise CxbwtError(st, self._what)  # cxbwt_last_error now holds the job's text
        return self.bwt, self.term

    def __del__(self):
        if self._h:  # never left running: wait (and drop the status)
            try:
                lib().cxbwt_job_wait(self._h, None)
            except Exception:
                pass


def _out_tensors(out, n_reads, n_bases, dev):
    import torch
    if out is not None:
        return out
    return (torch.empty(n_bases + n_reads, dtype=torch.uint8, device=dev),
            torch.empty(n_reads, dtype=torch.int64, device=dev))


def _opts(opts):
    """None, or (tile_items, chunk_items, schedule[, timing]) -> a cxbwt_opts pointer."""
    if opts is None:
        return None
    t, c, sched = opts[:3]
    return ctypes.byref(Opts(int(t), int(c), int(sched), int(opts[3]) if len(opts) > 3 else 0))


def build_start(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, workspace=None, out=None,
                stream=None, opts=None) -> BuildJob:
    """cxbwt_build_start: the build of `build`, returning at once (see BuildJob).
    opts: (tile_items, chunk_items, schedule[, timing]) for this build, else the thread's choices."""
    dev = packed.device
    if workspace is None:
        workspace = alloc_workspace(n_reads, n_bases, max_read_len, dev)
    bwt, term = _out_tensors(out, n_reads, n_bases, dev)
    h = ctypes.c_void_p()
    st = lib().cxbwt_build_start(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), n_reads,
                                 n_bases, max_read_len, ctypes.c_void_p(bwt.data_ptr()),
                                 ctypes.c_void_p(term.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel(), _opts(opts), _stream_ptr(stream), ctypes.byref(h))
    if st != OK:
        raise CxbwtError(st, "cxbwt_build_start")
    return BuildJob(h, "cxbwt_build_start", (packed, offsets, workspace), (bwt, term))


def build_batch_start(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, coll_reads, workspace=None,
                      out=None, stream=None, opts=None) -> BuildJob:
    """cxbwt_build_batch_start: the build of `build_batch`, returning at once (see BuildJob)."""
    import torch
    cr = np.ascontiguousarray(np.asarray(coll_reads, dtype=np.uint64))
    n_coll = cr.size - 1
    dev = packed.device
    if workspace is None:
        nbytes = batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll)
        if nbytes == 0:
            raise CxbwtError(ERANGE, "cxbwt_batch_workspace_bytes")
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    bwt, term = _out_tensors(out, n_reads, n_bases, dev)
    h = ctypes.c_void_p()
    st = lib().cxbwt_build_batch_start(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                       n_reads, n_bases, max_read_len, cr.ctypes.data_as(ctypes.c_void_p), n_coll,
                                       ctypes.c_void_p(bwt.data_ptr()), ctypes.c_void_p(term.data_ptr()),
                                       ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _opts(opts),
                                       _stream_ptr(stream), ctypes.byref(h))
    if st != OK:
        raise CxbwtError(st, "cxbwt_build_batch_start")
    return BuildJob(h, "cxbwt_build_batch_start", (packed, offsets, workspace), (bwt, term))


class BuildGraph:
    """A build captured once in a hipGraph and replayed (cxbwt_graph_*).

    The graph binds the given tensors: refill `packed` / `offsets` (same
    sizes, same bases per collection) and call run() (or launch() then
    finish()) for each build; the result lands in `bwt` / `term`.
    coll_reads: host read boundaries of the collections, or None for one.
    levels: sort levels scheduled inside the graph (0: enough for any input).
    """

    def __init__(self, packed, offsets, n_reads: int, n_bases: int, max_read_len: int, coll_reads=None,
                 levels: int = 0, workspace=None, out=None, stream=None):
        import torch
        dev = packed.device
        if coll_reads is None:
            cr = np.array([0, n_reads], dtype=np.uint64)
        else:
            cr = np.ascontiguousarray(np.asarray(coll_reads, dtype=np.uint64))
        n_coll = cr.size - 1
        if workspace is None:
            nbytes = batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll)
            if nbytes == 0:
                raise CxbwtError(ERANGE, "cxbwt_batch_workspace_bytes")
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        if out is None:
            out = (torch.empty(n_bases + n_reads, dtype=torch.uint8, device=dev),
                   torch.empty(n_reads, dtype=torch.int64, device=dev))
        self.packed, self.offsets, self.workspace = packed, offsets, workspace
        self.bwt, self.term = out
        self._h = ctypes.c_void_p()
        st = lib().cxbwt_graph_create(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                      n_reads, n_bases, max_read_len, cr.ctypes.data_as(ctypes.c_void_p), n_coll,
                                      ctypes.c_void_p(self.bwt.data_ptr()), ctypes.c_void_p(self.term.data_ptr()),
                                      ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), int(levels),
                                      _stream_ptr(stream), ctypes.byref(self._h))
        if st != OK:
            raise CxbwtError(st, "cxbwt_graph_create")

    def launch(self, stream=None) -> None:
        st = lib().cxbwt_graph_launch(self._h, _stream_ptr(stream))
        if st != OK:
            raise CxbwtError(st, "cxbwt_graph_launch")

    def finish(self, stream=None) -> None:
        st = lib().cxbwt_graph_finish(self._h, _stream_ptr(stream))
        if st != OK:
            raise CxbwtError(st, "cxbwt_graph_finish")

    def run(self, stream=None):
        self.launch(stream)
        self.finish(stream)
        return self.bwt, self.term

    def close(self) -> None:
        if self._h:
            lib().cxbwt_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def concat_collections(cols):
    """Host-side concatenation: (text, global offsets, coll_reads, max_read_len)."""
    texts = [np.asarray(c.text, dtype=np.uint8) for c in cols]
    text = np.concatenate(texts) if texts else np.zeros(0, np.uint8)
    offs = [np.zeros(1, dtype=np.uint64)]
    base = 0
    coll_reads = [0]
    maxlen = 0
    for c in cols:
        o = np.asarray(c.offsets, dtype=np.uint64)
        offs.append(o[1:] + np.uint64(base))
        base += int(o[-1])
        coll_reads.append(coll_reads[-1] + o.size - 1)
        if o.size > 1:
            maxlen = max(maxlen, int(np.max(np.diff(o.astype(np.int64)))))
    return text, np.concatenate(offs), np.array(coll_reads, dtype=np.uint64), maxlen


def split_batch_output(bwt: np.ndarray, term: np.ndarray, cols):
    """Per-collection (bwt, term_pos) views of a batch result (host arrays)."""
    out = []
    b0 = 0
    r0 = 0
    for c in cols:
        n, nb = c.n_reads, c.n_bases
        out.append((bwt[b0:b0 + n + nb], term[r0:r0 + n]))
        b0 += n + nb
        r0 += n
    return out


def build_batch_host(cols, device="cuda"):
    """Host collections in, per-collection host (bwt, term_pos) out."""
    import torch
    text, offsets, coll_reads, maxlen = concat_collections(cols)
    n = offsets.size - 1
    nb = int(offsets[-1])
    t_dev = torch.from_numpy(text).to(device) if nb else torch.empty(0, dtype=torch.uint8, device=device)
    o_dev = torch.from_numpy(offsets.view(np.int64)).to(device)
    packed, pstatus = pack(t_dev)
    bwt, term = build_batch(packed, o_dev, n, nb, maxlen, coll_reads)
    torch.cuda.synchronize()
    if int(pstatus.item()) != 0:
        raise CxbwtError(EDATA, "cxbwt_pack (non-ACGT byte)")
    return split_batch_output(bwt.cpu().numpy(), term.cpu().numpy().view(np.uint64), cols)


def last_error() -> str:
    """cxbwt_last_error: the text behind this thread's last EDEVICE / EDATA."""
    return lib().cxbwt_last_error().decode()


def last_stats() -> dict:
    s = Stats()
    lib().cxbwt_last_stats(ctypes.byref(s))
    return _stats_dict(s)


def _stats_dict(s) -> dict:
    out = {f: int(getattr(s, f)) for f, _ in Stats._fields_ if f not in ("ms", "launches")}
    out["ms"] = {k: float(s.ms[i]) for i, k in enumerate(KERNEL_CLASSES) if s.launches[i]}
    out["launches"] = {k: int(s.launches[i]) for i, k in enumerate(KERNEL_CLASSES) if s.launches[i]}
    return out


def set_tuning(tile_items: int, chunk_items: int) -> None:
    """Kernel instantiation used by later builds on this host thread."""
    st = lib().cxbwt_set_tuning(int(tile_items), int(chunk_items))
    if st != 0:
        raise CxbwtError(st, f"cxbwt_set_tuning({tile_items}, {chunk_items})")


def get_tuning() -> tuple:
    t, c = ctypes.c_uint32(), ctypes.c_uint32()
    st = lib().cxbwt_get_tuning(ctypes.byref(t), ctypes.byref(c))
    if st != 0:
        raise CxbwtError(st, "cxbwt_get_tuning")
    return int(t.value), int(c.value)


def set_schedule(schedule: int) -> None:
    """Sort schedule of later single-collection builds on this host thread."""
    st = lib().cxbwt_set_schedule(int(schedule))
    if st != 0:
        raise CxbwtError(st, f"cxbwt_set_schedule({schedule})")


def get_schedule() -> int:
    v = ctypes.c_uint32()
    st = lib().cxbwt_get_schedule(ctypes.byref(v))
    if st != 0:
        raise CxbwtError(st, "cxbwt_get_schedule")
    return int(v.value)


def set_timing(enable: bool) -> bool:
    """Per-kernel-class HIP-event timing of later builds on this host thread."""
    return bool(lib().cxbwt_set_timing(1 if enable else 0))


def build_host(text: np.ndarray, offsets: np.ndarray, max_read_len: int | None = None, device="cuda",
               max_range_suffixes: int | None = None, wide: bool = False):
    """Host arrays in, host arrays out: copy, pack and build on the device
    (in ranges of at most max_range_suffixes suffixes when given)."""
    import torch
    text = np.ascontiguousarray(text, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = offsets.size - 1
    nb = int(offsets[-1])
    if max_read_len is None:
        max_read_len = int(np.max(np.diff(offsets.astype(np.int64)))) if n else 0
    t_dev = torch.from_numpy(text).to(device) if nb else torch.empty(0, dtype=torch.uint8, device=device)
    o_dev = torch.from_numpy(offsets.view(np.int64)).to(device)
    packed, pstatus = pack(t_dev)
    if max_range_suffixes is None:
        bwt, term = build(packed, o_dev, n, nb, max_read_len)
    else:
        bwt, term = build_ranges(packed, o_dev, n, nb, max_read_len, max_range_suffixes, wide=wide)
    torch.cuda.synchronize()
    if int(pstatus.item()) != 0:
        raise CxbwtError(EDATA, "cxbwt_pack (non-ACGT byte)")
    return bwt.cpu().numpy(), term.cpu().numpy().view(np.uint64)
