"""Benchmark: multi-string BWT construction throughput on one MI355X.

A step is one pass of the whole device path over one resident collection:
pack the ASCII reads to 2-bit words, then cxbwt_build (suffix listing, the
digit levels, the in-workgroup sort + tie refinement, and the BWT emit).
The default workload is the plain single build of 4M reads x 100 bases from a
seeded 20 Mb random genome (20x coverage, 0.5% substitutions, both strands).

Prints one JSON line (rank 0): metric/value/unit, timing, the roofline of the
dominant kernel class (algorithmic bytes / its HIP-event time) and the CPU
oracle timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    "plain0": (0, "plain single build: 10k reads x 100 bp, 100 kb genome, 1% subst, both strands"),
    "plain1": (1, "plain single build: 4M reads x 100 bp, 20 Mb genome (20x), 0.5% subst, both strands"),
    "plain2": (2, "plain single build, repeat-heavy: 40M reads x 100 bp, 200 Mb genome with 10% 1-5 kb "
                  "repeat units x50 at 1% divergence, 0.5% subst"),
}


def algorithmic_bytes(stats: dict, n_reads: int, n_bases: int) -> dict:
    """Bytes each kernel class must move, by the per-suffix model of the design.

    gen          12.375 B/base: write 8 B key + 4 B handle, read 2-bit bases and end bits
    level_hist   8 B per suffix visit (key read) + 12 B per later-window fetch
    level_scan   4 B per tile counter, read and written (~0.25 B/suffix visit per pass)
    level_scatter 24 B per moved suffix: key + handle read and written
    local        13 B per suffix (key + handle read, 1 B BWT written) + 16 B per
                 later-window fetch (8 B of bases, 8 B of end bits) + 8 B per read start
    final_emit   13 B per suffix
    prep         17 B per read (two offsets, one BWT byte)
    """
    cs = stats.get("chunk_suffixes", 0)
    fin = n_bases - cs
    return {
        "prep": 17.0 * n_reads,
        "gen": 12.375 * n_bases,
        "level_hist": 8.0 * stats.get("level_suffixes", 0) + 12.0 * stats.get("regathered", 0),
        "level_scan": 2.0 * stats.get("level_suffixes", 0) / 4096 * 256 * 4 / 2,
        "level_scatter": 24.0 * stats.get("scattered_suffixes", 0),
        "local": 13.0 * cs + 16.0 * stats.get("window_fetches", 0) + 8.0 * n_reads,
        "final_emit": 13.0 * fin,
    }


def cpu_baseline(scale: float, threads: int) -> dict:
    from oracle import oracle  # the CPU baseline leg is the oracle itself
    from paper_1401_7457_amd import datagen
    col = datagen.plain_config(1, scale=scale)
    oracle.load()
    t0 = time.perf_counter()
    oracle.bwt(col.text, col.offsets, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": col.n_bases / dt / 1e9, "unit": "Gbases/s", "cores": threads, "kind": "oracle",
            "sample": f"same recipe at scale {scale:g}: {col.n_reads} reads x 100 bp from a "
                      f"{int(20_000_000 * scale)} b genome (same 20x coverage), {dt:.2f} s",
            "seconds": dt}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain1", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-scale", type=float, default=0.25, help="oracle sample: plain1 recipe at this scale")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this size (for counter calibration under rocprofv3)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1401_7457_amd import cxbwt, datagen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    cxbwt.lib()
    k, label = WORKLOADS[args.workload]
    col = datagen.plain_config(k)
    n, nb, maxlen = col.n_reads, col.n_bases, col.max_read_len
    print(f"[bench] workload {args.workload}: reads={n} bases={nb}", file=sys.stderr, flush=True)

    text = torch.from_numpy(col.text).cuda()
    offsets = torch.from_numpy(col.offsets.view(np.int64)).cuda()
    packed = torch.empty(cxbwt.packed_words(nb), dtype=torch.int64, device="cuda")
    pstatus = torch.empty(1, dtype=torch.int32, device="cuda")
    ws = cxbwt.alloc_workspace(n, nb, maxlen)
    bwt = torch.empty(nb + n, dtype=torch.uint8, device="cuda")
    term = torch.empty(n, dtype=torch.int64, device="cuda")

    def step():
        cxbwt.pack(text, out=packed, status=pstatus)
        cxbwt.build(packed, offsets, n, nb, maxlen, workspace=ws, out=(bwt, term))

    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if int(pstatus.item()) != 0:
        raise RuntimeError("input holds a non-ACGT byte")

    # timed region: whole steps, bracketed by synchronisation
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps

    # per-kernel-class timing (HIP events on the build's stream), separate steps
    cxbwt.set_timing(True)
    per_ms, per_launch, bytes_tot = {}, {}, {}
    stats = None
    tsteps = max(1, min(args.steps, 3))
    for _ in range(tsteps):
        step()
        stats = cxbwt.last_stats()
        for kname, v in stats["ms"].items():
            per_ms[kname] = per_ms.get(kname, 0.0) + v / tsteps
            per_launch[kname] = stats["launches"][kname]
    cxbwt.set_timing(False)
    torch.cuda.synchronize()
    model = algorithmic_bytes(stats, n, nb)
    dom = max(per_ms, key=per_ms.get)
    dom_ms = per_ms[dom]
    achieved = model[dom] / (dom_ms / 1e3) / 1e9
    model_total = sum(model.values())

    result = {
        "metric": "BWT build Gbases/s at 1 GPU",
        "value": nb / (ms_step / 1e3) / 1e9,
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": label, "reads": n, "bases": nb, "read_len": maxlen, "seed": col.seed,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_launch_ms": dom_ms / max(1, per_launch[dom]), "launches_per_step": per_launch[dom],
                     "algorithmic_bytes_per_step": model[dom]},
        "kernel_ms": per_ms,
        "model_bytes_per_base": model_total / nb,
        "hbm_frac_model_whole_step": model_total / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "build_stats": {kk: v for kk, v in stats.items() if kk not in ("ms", "launches")},
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        threads = len(os.sched_getaffinity(0))
        print(f"[bench] cpu baseline: oracle on {threads} threads", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.cpu_scale, threads)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
