"""Autotuner for the kernel instantiations of the library.

The library holds several instantiations of its level scatter (suffixes per
thread of a tile) and of its chunk kernel (suffixes per lane of a chunk); the
result is identical for all of them, only the speed differs.  `tune_build`
times each on the device for one input (after one warm-up build each) and
selects the fastest for later builds on the calling thread.  Choices are
remembered per workload shape (`shape_key`), so a serving loop tunes once per
shape class.
"""
from __future__ import annotations

import math

from . import cxbwt

_cache: dict = {}


def shape_key(n_reads: int, n_bases: int, max_read_len: int, n_coll: int = 1) -> tuple:
    """Shape class of a workload: size (power of 2), mean read length, read
    length bound, collections (power of 2)."""
    mean_len = n_bases // max(1, n_reads)
    return (max(0, int(math.log2(max(1, n_bases)))), int(mean_len // 25), int(max_read_len // 50),
            max(0, int(math.log2(max(1, n_coll)))))


def tune_build(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, coll_reads=None,
               repeats: int = 2, choices=None, workspace=None, out=None) -> dict:
    """Time every instantiation on this input and select the fastest.

    packed, offsets: device tensors as for `cxbwt.build`; coll_reads: host
    read boundaries for a batched build (None for one collection);
    workspace, out: the caller's buffers, else allocated here.  Returns
    {"choice": (tile_items, chunk_items), "ms": {choice: ms per build}}.
    """
    import torch
    choices = tuple(choices or cxbwt.TUNING_CHOICES)
    n_coll = 1 if coll_reads is None else len(coll_reads) - 1
    ws = workspace
    if ws is None and coll_reads is None:
        ws = cxbwt.alloc_workspace(n_reads, n_bases, max_read_len)
    elif ws is None:
        ws = torch.empty(cxbwt.batch_workspace_bytes(n_reads, n_bases, max_read_len, n_coll), dtype=torch.uint8,
                         device=packed.device)
    if out is None:
        out = (torch.empty(n_bases + n_reads, dtype=torch.uint8, device=packed.device),
               torch.empty(n_reads, dtype=torch.int64, device=packed.device))
    bwt, term = out

    def one():
        if coll_reads is None:
            cxbwt.build(packed, offsets, n_reads, n_bases, max_read_len, workspace=ws, out=(bwt, term))
        else:
            cxbwt.build_batch(packed, offsets, n_reads, n_bases, max_read_len, coll_reads, workspace=ws,
                              out=(bwt, term))

    before = cxbwt.get_tuning()
    times = {}
    try:
        for ch in choices:
            cxbwt.set_tuning(*ch)
            one()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(repeats):
                one()
            e1.record()
            torch.cuda.synchronize()
            times[ch] = e0.elapsed_time(e1) / repeats
    except Exception:
        cxbwt.set_tuning(*before)
        raise
    best = min(times, key=times.get)
    cxbwt.set_tuning(*best)
    _cache[shape_key(n_reads, n_bases, max_read_len, n_coll)] = best
    return {"choice": best, "ms": times}


def select_for(n_reads: int, n_bases: int, max_read_len: int, n_coll: int = 1) -> tuple | None:
    """Select the remembered choice for this shape class, if any (returns it)."""
    best = _cache.get(shape_key(n_reads, n_bases, max_read_len, n_coll))
    if best is not None:
        cxbwt.set_tuning(*best)
    return best
