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


def algorithmic_bytes(stats: dict, n_reads: int, n_bases: int, tile_len: int = 2048) -> dict:
    """Bytes each kernel class must move, by the per-suffix model of the design.

    gen           0.375 B per base: read the 2-bit bases and the end bits
                  (level 1 counts keys computed from the reads)
    level_hist    8 B per suffix visit (key read) + 12 B per later-window re-key
    level_scan    4 B per tile counter read and written (1 KB per tile of tile_len suffixes)
    level_scatter level 1: 12.375 B per base (bases + end bits read, key + handle
                  written); later levels: 24 B per moved suffix (key + handle
                  read and written)
    local         13 B per suffix (key + handle read, 1 B BWT written) + 16 B per
                  later-window text read (bases and read starts) + 8 B per read
    final_emit    13 B per suffix
    prep          17 B per read (two offsets, one BWT byte) + 0.19 B per base
                  (end-bit ranks)
    """
    cs = stats.get("chunk_suffixes", 0)
    fin = n_bases - cs
    scattered = stats.get("scattered_suffixes", 0)
    level1 = n_bases if stats.get("levels", 0) >= 1 and scattered >= n_bases else 0
    return {
        "prep": 17.0 * n_reads + 0.1875 * n_bases,
        "gen": 0.375 * n_bases,
        "level_hist": 8.0 * stats.get("level_suffixes", 0) - 8.0 * level1 + 12.0 * stats.get("regathered", 0),
        "level_scan": 2.0 * 1024 * stats.get("level_suffixes", 0) / tile_len,
        "level_scatter": 12.375 * level1 + 24.0 * (scattered - level1),
        "local": 13.0 * cs + 16.0 * stats.get("window_fetches", 0) + 8.0 * n_reads,
        "final_emit": 13.0 * fin,
    }


KERNELS_OF_CLASS = {
    "prep": ["k_prep", "k_text_records", "k_rank_count", "k_rank_top", "k_rank_words"],
    "gen": ["k_gen_hist", "k_gen"],
    "level_hist": ["k_level_hist"],
    "level_scan": ["k_group_scan", "k_level_scan"],
    "level_scatter": ["k_gen_scatter", "k_level_scatter"],
    "local": ["k_local"],
    "final_emit": ["k_emit_final", "k_term"],
}


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("cxbwt.hip", "device_common.h"):
        with open(os.path.join(ROOT, "paper_1401_7457_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kclass: str, launches_per_build: int, tuning: str):
    """HBM bytes per launch of a kernel class from the committed counter runs.

    None when no counter run exists for this workload, or when the kernel
    sources differ from the runs' or no run used the kernel instantiation
    (tuning, "AxB").
    The chunk kernel's work depends only on the chunk size (B): the level
    tile (A) cuts the levels' tiles, not the buckets that become chunks, so
    for that class only B has to match.
    """
    import json as _json
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = _json.load(open(path))
    if rec.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None
    # the main run, then counter runs of other instantiations of the same sources
    runs = [rec] + list(rec.get("other_tunings", []))

    def matches(run_tuning: str) -> bool:
        if kclass == "local":
            return run_tuning.split("x")[-1] == tuning.split("x")[-1]
        return run_tuning == tuning

    run = next((r for r in runs if r.get("tuning") == tuning), None) \
        or next((r for r in runs if matches(r.get("tuning") or "")), None)
    if run is None:
        return None
    tot = 0.0
    for k in KERNELS_OF_CLASS.get(kclass, []):
        e = run["kernels"].get(k)
        if e:
            tot += (e["fetch_MB_per_dispatch"] + e["write_MB_per_dispatch"]) * 1e6 * e["dispatches_per_build"]
    return tot / max(1, launches_per_build) if tot else None


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


def _batch_mode(args) -> dict:
    """Many collections: one batched build per wave against one build per collection."""
    import numpy as np
    import torch

    from paper_1401_7457_amd import cxbwt, datagen, serve
    cols = datagen.batch_collections(count=args.batch_count, scale=args.scale)
    sizes = [(c.n_reads, c.n_bases) for c in cols]
    waves = serve.plan_waves(sizes, budget_bytes=int(args.budget_gb * 2 ** 30))
    total = sum(nb for _, nb in sizes)
    print(f"[bench] batch: {len(cols)} collections, {total} bases, {len(waves)} wave(s)", file=sys.stderr,
          flush=True)
    dev = [(torch.from_numpy(c.text).cuda(), torch.from_numpy(c.offsets.view(np.int64)).cuda()) for c in cols]

    # each wave's reads laid end to end in HBM once, before any timing (the
    # inputs of a timed step are resident, as for the single build)
    wave_in = []
    for w in waves:
        parts = [torch.zeros(1, dtype=torch.int64, device="cuda")]
        base = 0
        for i in w:
            parts.append(dev[i][1][1:] + base)
            base += cols[i].n_bases
        cr = np.concatenate([[0], np.cumsum([cols[i].n_reads for i in w])]).astype(np.uint64)
        wave_in.append((torch.cat([dev[i][0] for i in w]), torch.cat(parts), cr, base,
                        max(cols[i].max_read_len for i in w)))
    torch.cuda.synchronize()

    def batched():
        for text, offs, cr, base, maxlen in wave_in:
            packed, _ = cxbwt.pack(text)
            cxbwt.build_batch(packed, offs, int(cr[-1]), base, maxlen, cr)

    def sequential():
        for i, c in enumerate(cols):
            packed, _ = cxbwt.pack(dev[i][0])
            cxbwt.build(packed, dev[i][1], c.n_reads, c.n_bases, c.max_read_len)

    tuning = None
    if not args.no_tune:
        # untimed: the instantiations are timed on the first wave, the fastest
        # kept for both forms
        from paper_1401_7457_amd import autotune
        text, offs, cr, base, maxlen = wave_in[0]
        packed, _ = cxbwt.pack(text)
        res = autotune.tune_build(packed, offs, int(cr[-1]), base, maxlen,
                                  coll_reads=cr, repeats=1)
        tuning = {"tile_items": res["choice"][0], "chunk_items": res["choice"][1],
                  "ms_per_choice": {f"{a}x{b}": round(v, 3) for (a, b), v in res["ms"].items()}}
        del packed

    out = {}
    for name, fn in (("batched", batched), ("one_at_a_time", sequential)):
        fn()  # warm-up (allocator, code objects)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        out[name] = {"seconds": dt, "gbases_per_s": total / dt / 1e9}

    # the same batch captured once in a hipGraph (levels scheduled on the
    # device, no host wait inside) and replayed into the captured buffers
    graph = None
    if len(waves) == 1:
        text, offs, cr, base, maxlen = wave_in[0]
        n_all = int(cr[-1])
        packed, _ = cxbwt.pack(text)
        eb, et = cxbwt.build_batch(packed, offs, n_all, base, maxlen, cr)
        levels = cxbwt.last_stats()["levels"]  # the device schedule covers what this input needs
        g = cxbwt.BuildGraph(packed, offs, n_all, base, maxlen, coll_reads=cr, levels=levels)

        def replay():
            cxbwt.pack(text, out=g.packed)
            g.run()

        replay()
        torch.cuda.synchronize()
        same = bool(torch.equal(g.bwt, eb) and torch.equal(g.term, et))
        t0 = time.perf_counter()
        for _ in range(args.steps):
            replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        graph = {"gbases_per_s": total / dt / 1e9, "levels_scheduled": levels, "equals_eager_build": same}
        g.close()
        del eb, et, packed
    return {
        "metric": "batched BWT build aggregate Gbases/s at 1 GPU",
        "value": out["batched"]["gbases_per_s"],
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": f"batched: {len(cols)} collections, log-uniform 5k-2M reads x{args.scale:g}, "
                               f"L in {{75,100,150}}, 1-10 Mb genomes x{args.scale:g}, 0.5% subst",
                   "bases": total, "waves": len(waves)},
        "one_at_a_time_gbases_per_s": out["one_at_a_time"]["gbases_per_s"],
        "speedup_vs_one_at_a_time": out["batched"]["gbases_per_s"] / out["one_at_a_time"]["gbases_per_s"],
        "graph_replay": graph,
        "tuning": tuning,
    }


def _serve_mode(args) -> dict:
    """Poisson job stream: continuous batching against one job at a time on the same trace."""
    import numpy as np
    import torch

    from paper_1401_7457_amd import cxbwt, datagen, serve
    jobs = datagen.job_stream(count=args.jobs, rate_per_s=1.0, scale=args.scale)
    mean_bases = float(np.mean([j.collection.n_bases for j in jobs]))
    # capacity: throughput of one-at-a-time builds of these jobs
    ex = serve.DeviceExecutor(keep_on_device=True)
    probe = jobs[: min(8, len(jobs))]
    rep0, _ = serve.replay([(0.0, j.collection) for j in probe], ex, int(args.budget_gb * 2 ** 30),
                           max_batch_jobs=1)
    capacity = rep0["gbases_per_s"] * 1e9  # bases per second
    rate = args.load * capacity / mean_bases
    arrivals = [(j.arrival_s / rate, j.collection) for j in jobs]
    total = sum(j.collection.n_bases for j in jobs)
    print(f"[bench] serve: {len(jobs)} jobs, {total} bases, rate {rate:.1f}/s (load {args.load})",
          file=sys.stderr, flush=True)
    res = {}
    for name, kw in (("continuous", {}), ("one_at_a_time", {"max_batch_jobs": 1})):
        torch.cuda.synchronize()
        rep, _ = serve.replay(arrivals, ex, int(args.budget_gb * 2 ** 30), **kw)
        res[name] = rep
    c, b = res["continuous"], res["one_at_a_time"]
    return {
        "metric": "served BWT build aggregate Gbases/s and p50/p99 job latency at 1 GPU",
        "value": c["gbases_per_s"],
        "unit": "Gbases/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": f"served: Poisson arrivals at {args.load:g} x measured capacity, {len(jobs)} jobs, "
                               f"log-uniform 10k-5M reads x{args.scale:g}, L uniform 100-250, 1% subst",
                   "bases": total, "budget_gb": args.budget_gb},
        "latency_note": "arrival to BWT complete on the device (device-to-host copy not included)",
        "latency_p50_s": c["latency_p50_s"],
        "latency_p99_s": c["latency_p99_s"],
        "mean_jobs_per_batch": c["mean_jobs_per_batch"],
        "one_at_a_time": {"gbases_per_s": b["gbases_per_s"], "latency_p50_s": b["latency_p50_s"],
                          "latency_p99_s": b["latency_p99_s"]},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve"],
                    help="plain: one collection (the headline line); batch / serve: the batched and served forms")
    ap.add_argument("--scale", type=float, default=0.05, help="batch/serve: size scale of the collections")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--jobs", type=int, default=60)
    ap.add_argument("--load", type=float, default=0.8, help="serve: offered load relative to measured capacity")
    ap.add_argument("--budget-gb", type=float, default=250.0)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain1", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-scale", type=float, default=0.1, help="oracle sample: plain1 recipe at this scale")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (it times every kernel instantiation on the workload before warm-up)")
    ap.add_argument("--tuning", default=None, help="force one instantiation, e.g. 8x6 (no autotuner)")
    ap.add_argument("--graph", action="store_true",
                    help="plain: also time replays of the build captured in a hipGraph (reported beside the line)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this size (for counter calibration under rocprofv3)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(one build runs on one device); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1401_7457_amd import cxbwt, datagen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    cxbwt.lib()
    if args.mode != "plain":
        res = _batch_mode(args) if args.mode == "batch" else _serve_mode(args)
        print(json.dumps(res), flush=True)
        return 0
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
        # a plain streaming kernel of known traffic (reads and writes
        # copy_calibration_mib MiB each) for scaling the HBM byte counters
        src = torch.ones((args.copy_calibration_mib << 20) // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    tuning = None
    if args.tuning:
        a, b = (int(v) for v in args.tuning.split("x"))
        cxbwt.set_tuning(a, b)
        tuning = {"tile_items": a, "chunk_items": b, "forced": True}
    elif not args.no_tune:
        # untimed: every instantiation is timed on this workload, the fastest kept
        from paper_1401_7457_amd import autotune
        cxbwt.pack(text, out=packed, status=pstatus)
        res = autotune.tune_build(packed, offsets, n, nb, maxlen, repeats=1, workspace=ws, out=(bwt, term))
        tuning = {"tile_items": res["choice"][0], "chunk_items": res["choice"][1],
                  "ms_per_choice": {f"{a}x{b}": round(v, 3) for (a, b), v in res["ms"].items()}}

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
    # the same build captured once in a hipGraph (levels sized and scheduled
    # on the device, as many as the eager build ran) and replayed: untimed
    # capture, then the same number of timed steps
    graph = None
    if args.graph:
        g = cxbwt.BuildGraph(packed, offsets, n, nb, maxlen, levels=stats["levels"], workspace=ws)

        def gstep():
            cxbwt.pack(text, out=packed, status=pstatus)
            g.run()

        for _ in range(max(1, args.warmup)):
            gstep()
        torch.cuda.synchronize()
        same = bool(torch.equal(g.bwt, bwt) and torch.equal(g.term, term))
        e2 = torch.cuda.Event(enable_timing=True)
        e3 = torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        for _ in range(args.steps):
            gstep()
        e3.record(stream)
        torch.cuda.synchronize()
        gms = e2.elapsed_time(e3) / args.steps
        graph = {"ms_per_step": gms, "gbases_per_s": nb / (gms / 1e3) / 1e9, "levels_scheduled": stats["levels"],
                 "equals_eager_build": same}
        g.close()

    model = algorithmic_bytes(stats, n, nb, tile_len=256 * cxbwt.get_tuning()[0])
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
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, dom, per_launch[dom],
                                                 "%dx%d" % cxbwt.get_tuning()),
                     "avg_launch_ms": dom_ms / max(1, per_launch[dom]), "launches_per_step": per_launch[dom],
                     "algorithmic_bytes_per_step": model[dom]},
        "kernel_ms": per_ms,
        "tuning": tuning,
        "model_bytes_per_base": model_total / nb,
        "hbm_frac_model_whole_step": model_total / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "build_stats": {kk: v for kk, v in stats.items() if kk not in ("ms", "launches")},
        "wall_s_timed": wall,
    }
    if graph is not None:
        result["graph_replay"] = graph
    if not args.no_cpu_baseline:
        threads = len(os.sched_getaffinity(0))
        print(f"[bench] cpu baseline: oracle on {threads} threads", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.cpu_scale, threads)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
