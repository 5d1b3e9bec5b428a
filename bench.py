"""Benchmark: multi-string BWT construction throughput on one MI355X.

A step is one pass of the whole device path over one resident collection:
pack the ASCII reads to 2-bit words, then cxbwt_build (suffix listing, the
digit levels, the in-workgroup sort + tie refinement, and the BWT emit).
The default workload (the headline line) is the largest single-GPU
configuration: the repeat-heavy plain build of 40M reads x 100 bases from a
seeded 200 Mb genome with 10% diverged repeat families (4 Gbases).  The
20x-coverage build of 4M reads x 100 bases (400 Mbases) follows as a
secondary line inside the same JSON object.

Prints one JSON line (rank 0): metric/value/unit, timing, the roofline of the
dominant kernel class (algorithmic bytes / its HIP-event time, with the HBM
traffic of the committed counter runs per launch and per step) and the CPU
oracle timed on a bounded sample of the same recipe on the host cores.

Other modes: --mode batch / serve (the batched and served forms) and
--mode sweep (100/200/400-base reads at equal total bases).
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
DIGIT_BITS = 8  # radix digit of every level (a wider one loses on its write pattern: --mode ceilings)

WORKLOADS = {
    "plain0": (0, "plain single build: 10k reads x 100 bp, 100 kb genome, 1% subst, both strands"),
    "plain1": (1, "plain single build: 4M reads x 100 bp, 20 Mb genome (20x), 0.5% subst, both strands"),
    "plain2": (2, "plain single build, repeat-heavy: 40M reads x 100 bp, 200 Mb genome with 10% 1-5 kb "
                  "repeat units x50 at 1% divergence, 0.5% subst, both strands"),
}
DEFAULT_WORKLOAD = "plain2"      # the largest configuration one GPU builds in one call
SECONDARY_WORKLOAD = "plain1"    # reported inside the same line
# oracle sample per headline workload: that recipe at this scale (10-30 s of CPU work)
CPU_SAMPLE_SCALE = {"plain0": 1.0, "plain1": 0.1, "plain2": 0.02}


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
    if stats.get("schedule", 0) == 1:
        # the stringword schedule: per window, keys computed in base order
        # (text record and start ranks ~1.25 B, key written 8 B) and permuted
        # by handle (handle 4 B, key 8 B gathered, key 8 B written); per digit
        # pass a histogram read (8 B) and a scatter (24 B); one emit (13 B)
        return {
            "prep": 17.0 * n_reads + 0.1875 * n_bases,
            "gen": 29.25 * stats.get("window_fetches", 0),
            "level_hist": 8.0 * stats.get("level_suffixes", 0),
            "level_scan": 2.0 * 1024 * stats.get("level_suffixes", 0) / 2048,
            "level_scatter": 24.0 * stats.get("scattered_suffixes", 0),
            "local": 0.0,
            "final_emit": 13.0 * n_bases,
        }
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

# the device code whose counter runs a traffic record holds (host code that
# only sequences launches is not part of it)
KERNEL_SOURCES = ("cxbwt_kernels.h", "device_common.h")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1401_7457_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(workload: str):
    """The committed counter-run record of a workload (profiles/<workload>_traffic.json),
    or None when there is none or it was taken with other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None
    return rec


def measured_traffic(workload: str, kclass: str, tuning: str):
    """HBM bytes per build (one step) of a kernel class from the committed counter runs.

    Each counter run holds, per kernel, the FETCH_SIZE and WRITE_SIZE totals
    (MB) over `builds` builds; they are scaled by the record's calibration
    (the same counters read for a plain copy of known size).  None when no
    record matches the kernel sources or no run used the kernel instantiation
    (tuning, "AxB").  The chunk kernel's work depends only on the chunk size
    (B): the level tile (A) cuts the levels' tiles, not the buckets that
    become chunks, so for that class only B has to match.
    """
    rec = traffic_record(workload)
    if rec is None:
        return None

    def matches(run_tuning: str) -> bool:
        if kclass == "local":
            return run_tuning.split("x")[-1] == tuning.split("x")[-1]
        return run_tuning == tuning

    runs = rec.get("runs", [])
    run = next((r for r in runs if r.get("tuning") == tuning), None) \
        or next((r for r in runs if matches(r.get("tuning") or "")), None)
    if run is None:
        return None
    cal = rec["calibration"]
    tot = 0.0
    for k in KERNELS_OF_CLASS.get(kclass, []):
        e = run["kernels"].get(k)
        if e:
            tot += (e["fetch_MB"] * cal["fetch_factor"] + e["write_MB"] * cal["write_factor"]) * 1e6
    return tot / rec["builds"] if tot else None


def host_info() -> dict:
    """CPU model, host RAM and the threads this process may use."""
    model, ram_gb = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    ram_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_ram_gib": ram_gb, "threads": len(os.sched_getaffinity(0))}


def cpu_baseline(workload: str, threads: int) -> dict:
    """The oracle (untuned) on the host cores: the headline recipe at a bounded
    scale on every thread, plus the 1 Mbase recipe (plain0) on every thread
    (median of 3) and on one thread."""
    from oracle import oracle  # the CPU baseline leg is the oracle itself
    from paper_1401_7457_amd import datagen
    k, _ = WORKLOADS[workload]
    scale = CPU_SAMPLE_SCALE[workload]
    col = datagen.plain_config(k, scale=scale)
    oracle.load()
    t0 = time.perf_counter()
    oracle.bwt(col.text, col.offsets, threads=threads)
    dt = time.perf_counter() - t0
    small = datagen.plain_config(0)
    runs = []
    for _ in range(3):
        t1 = time.perf_counter()
        oracle.bwt(small.text, small.offsets, threads=threads)
        runs.append(time.perf_counter() - t1)
    t1 = time.perf_counter()
    oracle.bwt(small.text, small.offsets, threads=1)
    one = time.perf_counter() - t1
    info = host_info()
    return {"value": col.n_bases / dt / 1e9, "unit": "Gbases/s", "cores": threads, "kind": "oracle",
            "sample": f"{workload} recipe at scale {scale:g}: {col.n_reads} reads x 100 bp, {col.n_bases} bases "
                      f"(genome and read count scaled together, same coverage), {dt:.2f} s",
            "seconds": dt, "cpu_model": info["cpu_model"], "host_ram_gib": info["host_ram_gib"],
            "plain0_seconds_median3": sorted(runs)[1], "plain0_seconds_1_thread": one,
            "plain0_gbases_per_s_1_thread": small.n_bases / one / 1e9}


SCHEDULE_NAMES = {0: "msd", 1: "stringword"}


def choice_name(ch) -> str:
    """"AxB" for an MSD choice, "AxB-stringword" for the stringword schedule."""
    a, b, sched = ch
    return f"{a}x{b}" + ("" if sched == 0 else "-" + SCHEDULE_NAMES[sched])


def tuning_record(res: dict, repeats: int) -> dict:
    a, b, sched = res["choice"]
    return {"tile_items": a, "chunk_items": b, "schedule": SCHEDULE_NAMES[sched], "digit_bits": DIGIT_BITS,
            "repeats": repeats, "ms_per_choice": {choice_name(ch): round(v, 3) for ch, v in res["ms"].items()}}


def _tune(args, packed, offsets, n, nb, maxlen, ws, bwt, term, pstatus, text):
    """Autotuner (untimed): every instantiation timed on this workload, the fastest kept."""
    from paper_1401_7457_amd import autotune, cxbwt
    if args.tuning:
        a, b = (int(v) for v in args.tuning.split("x")[:2])
        sched = cxbwt.SCHEDULE_STRINGWORD if args.tuning.endswith("sw") else cxbwt.SCHEDULE_MSD
        autotune.apply((a, b, sched))
        return {"tile_items": a, "chunk_items": b, "schedule": SCHEDULE_NAMES[sched], "digit_bits": DIGIT_BITS,
                "forced": True}
    if args.no_tune:
        return None
    cxbwt.pack(text, out=packed, status=pstatus)
    res = autotune.tune_build(packed, offsets, n, nb, maxlen, repeats=args.tune_repeats, workspace=ws,
                              out=(bwt, term))
    return tuning_record(res, args.tune_repeats)


def _plain_line(args, workload: str, col=None, label: str | None = None) -> dict:
    """One resident collection: timed steps, per-class kernel times, the roofline."""
    import numpy as np
    import torch

    from paper_1401_7457_amd import cxbwt, datagen
    if col is None:
        k, label = WORKLOADS[workload]
        col = datagen.plain_config(k)
    n, nb, maxlen = col.n_reads, col.n_bases, col.max_read_len
    print(f"[bench] workload {workload}: reads={n} bases={nb}", file=sys.stderr, flush=True)

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

    tuning = _tune(args, packed, offsets, n, nb, maxlen, ws, bwt, term, pstatus, text)
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

    # per-kernel-class timing (HIP events the library records on the build's
    # stream, which is torch's current stream here), separate steps
    cxbwt.set_timing(True)
    per_ms, per_launch = {}, {}
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

    graph = None
    if args.graph:
        # the same build captured once in a hipGraph (levels sized and
        # scheduled on the device, as many as the eager build ran) and
        # replayed: untimed capture, then the same number of timed steps
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

    tuning_str = "%dx%d" % cxbwt.get_tuning()
    model = algorithmic_bytes(stats, n, nb, tile_len=256 * cxbwt.get_tuning()[0])
    dom = max(per_ms, key=per_ms.get)
    dom_ms = per_ms[dom]
    launches = max(1, per_launch[dom])
    alg_step = model[dom]
    achieved = alg_step / (dom_ms / 1e3) / 1e9  # = per-launch bytes / average launch time
    traffic_step = measured_traffic(workload, dom, tuning_str)
    rec = traffic_record(workload)
    roofline = {
        "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": None if traffic_step is None else traffic_step / launches,
        "traffic_per_step": traffic_step,
        "algorithmic_bytes_per_launch": alg_step / launches,
        "algorithmic_bytes_per_step": alg_step,
        "traffic_ratio": None if traffic_step is None else traffic_step / alg_step,
        "kernel_ms_per_step": dom_ms, "launches_per_step": per_launch[dom], "avg_launch_ms": dom_ms / launches,
        "traffic_calibration": None if rec is None else rec["calibration"].get("note"),
    }
    model_total = sum(model.values())
    return {
        "value": nb / (ms_step / 1e3) / 1e9,
        "ms_per_step": ms_step,
        "config": {"workload": label, "reads": n, "bases": nb, "read_len": maxlen, "seed": col.seed,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "kernel_ms": per_ms,
        "tuning": tuning,
        "model_bytes_per_base": model_total / nb,
        "hbm_frac_model_whole_step": model_total / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "build_stats": {kk: v for kk, v in stats.items() if kk not in ("ms", "launches")},
        "wall_s_timed": wall,
        "graph_replay": graph,
    }


def _sweep_mode(args) -> dict:
    """Read-length sweep at equal total bases (Section 4.3, Table 4: 100/200/400 bp)."""
    import gc

    import torch

    from paper_1401_7457_amd import datagen
    total = int(args.sweep_gbases * 1e9)
    lines = []
    for L in (100, 200, 400):
        col = datagen.length_sweep_config(L, total)
        label = f"read-length sweep: {col.n_reads} reads x {L} bp ({total / 1e9:g} Gbases), " \
                f"{total // 20 / 1e6:g} Mb genome (20x), 0.5% subst, both strands"
        line = _plain_line(args, f"sweep{L}", col=col, label=label)
        line["read_len"] = L
        lines.append(line)
        print(f"[bench] sweep {L} bp: {line['ms_per_step']:.1f} ms/step", file=sys.stderr, flush=True)
        del col
        gc.collect()
        torch.cuda.empty_cache()
    base = lines[0]["value"]
    return {
        "metric": "BWT build Gbases/s at 1 GPU by read length (equal total bases)",
        "value": base,
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": f"read-length sweep at {total / 1e9:g} Gbases: 100/200/400 bp"},
        "lines": [{"read_len": x["read_len"], "gbases_per_s": x["value"], "ms_per_step": x["ms_per_step"],
                   "relative_to_100bp": x["value"] / base, "hbm_frac_model_whole_step": x["hbm_frac_model_whole_step"],
                   "model_bytes_per_base": x["model_bytes_per_base"], "kernel_ms": x["kernel_ms"],
                   "tuning": x["tuning"], "build_stats": x["build_stats"], "config": x["config"]} for x in lines],
    }


def _ranges_mode(args) -> dict:
    """The 4 Gbase build in key ranges (Section 3.1, Fig. 2): budgets of about
    1/2, 1/4 and 1/8 of its suffixes, against the build of all of it at once
    (the same instantiation): ms per step, ranges, workspace, and whether the
    output equals the build's."""
    import hashlib

    import numpy as np
    import torch

    from paper_1401_7457_amd import autotune, cxbwt, datagen
    k, label = WORKLOADS[args.workload]
    col = datagen.plain_config(k)
    n, nb, maxlen = col.n_reads, col.n_bases, col.max_read_len
    print(f"[bench] ranges: {args.workload} reads={n} bases={nb}", file=sys.stderr, flush=True)
    text = torch.from_numpy(col.text).cuda()
    offsets = torch.from_numpy(col.offsets.view(np.int64)).cuda()
    packed, _ = cxbwt.pack(text)
    bwt = torch.empty(nb + n, dtype=torch.uint8, device="cuda")
    term = torch.empty(n, dtype=torch.int64, device="cuda")
    if args.tuning:
        a, b = (int(v) for v in args.tuning.split("x")[:2])
        autotune.apply((a, b, cxbwt.SCHEDULE_MSD))

    def digest():
        return hashlib.sha256(bwt.cpu().numpy().tobytes() + term.cpu().numpy().tobytes()).hexdigest()[:16]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ws = cxbwt.alloc_workspace(n, nb, maxlen)
    ms_all = timed(lambda: cxbwt.build(packed, offsets, n, nb, maxlen, workspace=ws, out=(bwt, term)))
    ref = digest()
    ws_all = ws.numel()
    del ws
    torch.cuda.empty_cache()
    lines = [{"ranges": 1, "budget_suffixes": nb, "ms_per_step": ms_all, "gbases_per_s": nb / ms_all / 1e6,
              "workspace_bytes": ws_all, "same_output": True, "form": "cxbwt_build"}]
    for parts in (2, 4, 8):
        m = nb // parts + 1
        wsb = cxbwt.range_workspace_bytes(n, nb, maxlen, m)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        ms = timed(lambda: cxbwt.build_ranges(packed, offsets, n, nb, maxlen, m, workspace=ws, out=(bwt, term)))
        st = cxbwt.last_stats()
        lines.append({"ranges": st["ranges"], "budget_suffixes": m, "ms_per_step": ms, "gbases_per_s": nb / ms / 1e6,
                      "workspace_bytes": wsb, "same_output": digest() == ref, "form": "cxbwt_build_ranges"})
        print(f"[bench] ranges budget {m}: {st['ranges']} ranges, {ms:.1f} ms/step", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    return {
        "metric": "BWT build Gbases/s at 1 GPU in key ranges", "value": lines[-1]["gbases_per_s"], "unit": "Gbases/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "data": "synthetic",
        "config": {"workload": label, "reads": n, "bases": nb, "tuning": "x".join(map(str, cxbwt.get_tuning()))},
        "lines": lines,
    }


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
                                  coll_reads=cr, repeats=args.tune_repeats)
        tuning = tuning_record(res, args.tune_repeats)
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
    # the client receives each job's reads into pinned host memory (prepared
    # before the trace starts), so the server's staging copy is asynchronous
    for j in jobs:
        c = j.collection
        j.collection = datagen.Collection(torch.from_numpy(c.text).pin_memory(), c.offsets, c.seed, c.label)
    budget = int(args.budget_gb * 2 ** 30)
    ex = serve.DeviceExecutor(keep_on_device=True)
    # capacity: one-at-a-time builds of the first jobs, measured warm (the
    # probe runs twice; the second run is kept)
    probe = [(0.0, j.collection) for j in jobs[: min(8, len(jobs))]]
    for _ in range(2):
        rep0, _ = serve.replay(probe, ex, budget, max_batch_jobs=1, max_inflight=1)
    capacity = rep0["gbases_per_s"] * 1e9  # bases per second
    rate = args.load * capacity / mean_bases
    arrivals = [(j.arrival_s / rate, j.collection) for j in jobs]
    total = sum(j.collection.n_bases for j in jobs)
    print(f"[bench] serve: {len(jobs)} jobs, {total} bases, capacity {capacity / 1e9:.2f} Gbases/s, "
          f"rate {rate:.1f}/s (load {args.load})", file=sys.stderr, flush=True)
    res = {}
    for name, kw in (("continuous", {"max_inflight": 2}), ("one_at_a_time", {"max_batch_jobs": 1, "max_inflight": 1})):
        torch.cuda.synchronize()
        rep, _ = serve.replay(arrivals, ex, budget, **kw)
        res[name] = rep
        print(f"[bench] serve {name}: {rep['gbases_per_s']:.2f} Gbases/s, p50 {rep['latency_p50_s'] * 1e3:.1f} ms, "
              f"p99 {rep['latency_p99_s'] * 1e3:.1f} ms, {rep['mean_jobs_per_batch']:.2f} jobs per batch",
              file=sys.stderr, flush=True)
    c, b = res["continuous"], res["one_at_a_time"]
    return {
        "metric": "served BWT build aggregate Gbases/s and p50/p99 job latency at 1 GPU",
        "value": c["gbases_per_s"],
        "unit": "Gbases/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "config": {"workload": f"served: Poisson arrivals at {args.load:g} x measured capacity, {len(jobs)} jobs, "
                               f"reads in pinned host memory, up to 2 batches building at once, "
                               f"log-uniform 10k-5M reads x{args.scale:g}, L uniform 100-250, 1-10 Mb genomes "
                               f"x{args.scale:g}, 1% subst",
                   "bases": total, "budget_gb": args.budget_gb, "mean_job_bases": mean_bases},
        "capacity_one_at_a_time_gbases_per_s": capacity / 1e9,
        "offered_rate_jobs_per_s": rate,
        "latency_note": "arrival to BWT complete on the device (device-to-host copy not included)",
        "latency_p50_s": c["latency_p50_s"],
        "latency_p99_s": c["latency_p99_s"],
        "mean_jobs_per_batch": c["mean_jobs_per_batch"],
        "batches": c["batches"],
        "makespan_s": c["makespan_s"],
        "one_at_a_time": {"gbases_per_s": b["gbases_per_s"], "latency_p50_s": b["latency_p50_s"],
                          "latency_p99_s": b["latency_p99_s"], "makespan_s": b["makespan_s"]},
        "speedup_vs_one_at_a_time": c["gbases_per_s"] / b["gbases_per_s"],
    }


def _ceilings_mode(args) -> dict:
    """Memory-system ceilings the kernels are measured against, with torch's own
    kernels (torch's, and one gather kernel of this package): a streaming
    copy, random 16-byte gathers (the window fetches' access pattern) and
    32-byte ones (two windows a load), and writes in runs of consecutive records per bucket per
    tile (the level scatters' write pattern, for 256 buckets and for the
    wider digits a 10- or 12-bit digit would give; index_copy_ also reads its
    8-byte indices), each timed with events over several repetitions."""
    import torch
    out = {}
    reps = max(3, args.steps)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    n = 1 << 28  # 2 GiB of int64
    src = torch.ones(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src))
    out["copy_gb_per_s"] = 2 * 8 * n / t / 1e9
    del src, dst
    # random row gathers with the library's measurement kernel (hashed
    # indices, four loads in flight per thread, 2^26 loads a launch)
    import ctypes
    cl = ctypes.CDLL(os.path.join(ROOT, "paper_1401_7457_amd", "libcxbwt_ceilings.so"))
    cl.cxbwt_ceiling_gather.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    cl.cxbwt_ceiling_gather.restype = ctypes.c_int
    table = torch.zeros(8 << 30, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    n_loads = 1 << 26
    for table_mib, row_bytes in ((256, 16), (4096, 16), (8192, 16), (4096, 32), (8192, 32)):
        rows = (table_mib << 20) // row_bytes
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

        def gather():
            rc = cl.cxbwt_ceiling_gather(ctypes.c_void_p(table.data_ptr()), rows, row_bytes, n_loads, 14017457,
                                         ctypes.c_void_p(sink.data_ptr()), stream)
            if rc != 0:
                raise RuntimeError(f"cxbwt_ceiling_gather: {rc}")
        t = timed(gather)
        out[f"random_{row_bytes}B_loads_per_s_table_{table_mib}MiB"] = n_loads / t
    del table, sink
    # the write pattern of a level scatter: ~400M (key u64, handle u32)
    # records in tiles of nb * r, each tile writing a run of r records to
    # each of nb evenly filled buckets at the bucket's running position.  The
    # 8-bit digit of the library is nb = 256 (runs of 16 for its 4096-suffix
    # tile); a 10-bit digit over the same tile would write runs of 4 to 1024
    # buckets, over a tile twice as long runs of 8.
    for nbk, r in ((256, 8), (256, 16), (1024, 4), (1024, 8), (4096, 2)):
        ntiles = 400_000_000 // (nbk * r)
        t_ = torch.arange(ntiles, device="cuda").view(-1, 1, 1)
        b_ = torch.arange(nbk, device="cuda").view(1, -1, 1)
        k_ = torch.arange(r, device="cuda").view(1, 1, -1)
        pos = (b_ * (ntiles * r) + t_ * r + k_).reshape(-1)
        m = pos.numel()
        keys = torch.ones(m, dtype=torch.int64, device="cuda")
        hdl = torch.ones(m, dtype=torch.int32, device="cuda")
        ko = torch.empty_like(keys)
        ho = torch.empty_like(hdl)

        def scat():
            ko.index_copy_(0, pos, keys)
            ho.index_copy_(0, pos, hdl)
        t = timed(scat)
        name = f"scatter_runs_of_{r}" if nbk == 256 else f"scatter_{nbk}_buckets_runs_of_{r}"
        out[f"{name}_ms_per_400M"] = t * 1e3 * 400_000_000 / m
        out[f"{name}_gb_per_s"] = m * 24 / t / 1e9
        del pos, keys, hdl, ko, ho, t_, b_, k_
    return {"metric": "memory-system ceilings at 1 GPU", "unit": "various", "n_gpus": 1,
            "data": "synthetic", "reps": reps, "ceilings": out}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", default="plain", choices=["plain", "batch", "serve", "sweep", "ceilings", "ranges"],
                    help="plain: one collection (the headline line); batch / serve: the batched and served forms; "
                         "sweep: 100/200/400-base reads at equal total bases; ranges: the --workload build in "
                         "1/2/4/8 key ranges")
    ap.add_argument("--scale", type=float, default=0.05, help="batch/serve: size scale of the collections")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--jobs", type=int, default=60)
    ap.add_argument("--load", type=float, default=1.5,
                    help="serve: offered load relative to the measured one-at-a-time capacity")
    ap.add_argument("--budget-gb", type=float, default=250.0)
    ap.add_argument("--sweep-gbases", type=float, default=2.0, help="sweep: total bases per read length")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-secondary", action="store_true",
                    help=f"plain: skip the {SECONDARY_WORKLOAD} line reported beside the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (it times every kernel instantiation on the workload before warm-up)")
    ap.add_argument("--tune-repeats", type=int, default=3, help="timed builds per instantiation in the autotuner")
    ap.add_argument("--tuning", default=None,
                    help="force one choice, e.g. 8x6, or 8x6sw for the stringword schedule (no autotuner)")
    ap.add_argument("--graph", action="store_true",
                    help="plain: also time replays of the build captured in a hipGraph (reported beside the line)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run, before the builds, one device copy of this size and one random gather of "
                         "16-byte rows from a table of this size (for counter calibration under rocprofv3)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(one build runs on one device); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_1401_7457_amd import cxbwt

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    cxbwt.lib()
    if args.copy_calibration_mib:
        calibration_kernels(args.copy_calibration_mib)
    if args.mode in ("batch", "serve", "sweep", "ceilings", "ranges"):
        res = {"batch": _batch_mode, "serve": _serve_mode, "sweep": _sweep_mode,
               "ceilings": _ceilings_mode, "ranges": _ranges_mode}[args.mode](args)
        print(json.dumps(res), flush=True)
        return 0

    head = _plain_line(args, args.workload)
    result = {
        "metric": "BWT build Gbases/s at 1 GPU",
        "value": head["value"],
        "unit": "Gbases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
    }
    result.update({k: v for k, v in head.items() if k not in ("value", "ms_per_step", "graph_replay")})
    if head["graph_replay"] is not None:
        result["graph_replay"] = head["graph_replay"]
    if args.workload != SECONDARY_WORKLOAD and not args.no_secondary:
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        sec = _plain_line(args, SECONDARY_WORKLOAD)
        result["secondary"] = {"workload": sec["config"]["workload"], "gbases_per_s": sec["value"],
                               "ms_per_step": sec["ms_per_step"], "config": sec["config"],
                               "roofline": sec["roofline"], "kernel_ms": sec["kernel_ms"], "tuning": sec["tuning"],
                               "model_bytes_per_base": sec["model_bytes_per_base"],
                               "hbm_frac_model_whole_step": sec["hbm_frac_model_whole_step"],
                               "build_stats": sec["build_stats"]}
        if sec["graph_replay"] is not None:
            result["secondary"]["graph_replay"] = sec["graph_replay"]
    if not args.no_cpu_baseline:
        threads = len(os.sched_getaffinity(0))
        print(f"[bench] cpu baseline: oracle on {threads} threads", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.workload, threads)
    print(json.dumps(result), flush=True)
    return 0


def calibration_kernels(mib: int) -> None:
    """Kernels of known traffic for scaling the HBM byte counters: torch's neg
    over `mib` MiB (reads and writes `mib` MiB each), then an index_select of
    16-byte rows at uniform random indices from a table of `mib` MiB (one
    random 16-byte load per output row, rows = table rows / 4; the indices
    are read and the rows written in order)."""
    import torch
    src = torch.ones((mib << 20) // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    table = torch.zeros(((mib << 20) // 16, 2), dtype=torch.int64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(14017457)
    idx = torch.randint(0, table.shape[0], (table.shape[0] // 4,), device="cuda", generator=g)
    torch.cuda.synchronize()
    out = table.index_select(0, idx)
    torch.cuda.synchronize()
    print(f"[bench] calibration: neg over {mib} MiB; index_select of {idx.numel()} random 16-byte rows "
          f"from {table.shape[0]} rows", file=sys.stderr, flush=True)
    del table, idx, out


if __name__ == "__main__":
    sys.exit(main())
