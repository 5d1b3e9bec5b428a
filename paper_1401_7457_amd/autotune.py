"""Autotuner for the kernel instantiations and the sort schedule of the library.

The library holds several instantiations of its level scatter (suffixes per
thread of a tile) and of its chunk kernel (suffixes per lane of a chunk), and
two sort schedules for a single collection: most significant digit first with
tie refinement (the default) and the paper's stringword schedule (LSD passes
over every window).  The result is identical for all of them; only the speed
differs.  `tune_build` times each choice on the device for one input (one
warm-up build, then `repeats` timed builds, the median kept) and selects the
fastest for later builds on the calling thread.  Choices are remembered per
workload shape (`shape_key`) in memory and in a JSON file
($CXBWT_TUNE_CACHE, default ~/.cache/cxbwt/tuning.json), so a serving loop or
a later process tunes once per shape class.
"""
from __future__ import annotations

import json
import math
import os

from . import cxbwt

_cache: dict = {}


def cache_path() -> str:
    return os.environ.get("CXBWT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cxbwt", "tuning.json"))


def choices_for(n_coll: int = 1) -> tuple:
    """(tile_items, chunk_items, schedule) choices: every instantiation with the
    MSD schedule, and for one collection the stringword schedule (its passes do
    not depend on the instantiation)."""
    out = tuple((t, c, cxbwt.SCHEDULE_MSD) for t, c in cxbwt.TUNING_CHOICES)
    if n_coll == 1:
        out += ((cxbwt.TUNING_CHOICES[0][0], cxbwt.TUNING_CHOICES[0][1], cxbwt.SCHEDULE_STRINGWORD),)
    return out


def shape_key(n_reads: int, n_bases: int, max_read_len: int, n_coll: int = 1) -> tuple:
    """Shape class of a workload: size (power of 2), mean read length, read
    length bound, collections (power of 2)."""
    mean_len = n_bases // max(1, n_reads)
    return (max(0, int(math.log2(max(1, n_bases)))), int(mean_len // 25), int(max_read_len // 50),
            max(0, int(math.log2(max(1, n_coll)))))


def _key_str(key: tuple) -> str:
    return "_".join(str(v) for v in key)


def apply(choice) -> None:
    """Select a (tile_items, chunk_items, schedule) choice for this thread."""
    t, c, sched = choice
    cxbwt.set_tuning(t, c)
    cxbwt.set_schedule(sched)


def current() -> tuple:
    return (*cxbwt.get_tuning(), cxbwt.get_schedule())


def _load_file() -> dict:
    try:
        with open(cache_path()) as f:
            return {k: tuple(v) for k, v in json.load(f).items()}
    except (OSError, ValueError):
        return {}


def _save_file(key: tuple, choice: tuple) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        data = _load_file()
        data[_key_str(key)] = list(choice)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump({k: list(v) for k, v in data.items()}, f)
        os.replace(tmp, path)
    except OSError:
        pass  # the in-memory cache still holds the choice


def tune_build(packed, offsets, n_reads: int, n_bases: int, max_read_len: int, coll_reads=None,
               repeats: int = 3, choices=None, workspace=None, out=None, persist: bool = True) -> dict:
    """Time every choice on this input and select the fastest.

    packed, offsets: device tensors as for `cxbwt.build`; coll_reads: host
    read boundaries for a batched build (None for one collection);
    workspace, out: the caller's buffers, else allocated here.  Returns
    {"choice": (tile_items, chunk_items, schedule), "ms": {choice: median ms
    per build}}.
    """
    import torch
    n_coll = 1 if coll_reads is None else len(coll_reads) - 1
    choices = tuple(choices or choices_for(n_coll))
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

    before = current()
    times = {}
    try:
        for ch in choices:
            apply(ch)
            one()
            torch.cuda.synchronize()
            runs = []
            for _ in range(max(1, repeats)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                one()
                e1.record()
                torch.cuda.synchronize()
                runs.append(e0.elapsed_time(e1))
            times[ch] = sorted(runs)[len(runs) // 2]
    except Exception:
        apply(before)
        raise
    best = min(times, key=times.get)
    apply(best)
    key = shape_key(n_reads, n_bases, max_read_len, n_coll)
    _cache[key] = best
    if persist:
        _save_file(key, best)
    return {"choice": best, "ms": times}


def remembered(n_reads: int, n_bases: int, max_read_len: int, n_coll: int = 1) -> tuple | None:
    """The remembered (tile_items, chunk_items, schedule) choice for this
    shape class, if any; selects nothing (pass it as a started build's opts)."""
    key = shape_key(n_reads, n_bases, max_read_len, n_coll)
    best = _cache.get(key)
    if best is None:
        best = _load_file().get(_key_str(key))
        if best is not None and len(best) != 3:
            best = None  # written before the schedule was a choice
        if best is not None:
            _cache[key] = best
    return best


def select_for(n_reads: int, n_bases: int, max_read_len: int, n_coll: int = 1) -> tuple | None:
    """Select the remembered choice for this shape class on this thread, if any (returns it)."""
    best = remembered(n_reads, n_bases, max_read_len, n_coll)
    if best is not None:
        apply(best)
    return best
