"""Host logic of bench.py: the one-GPU refusal, the byte model and the
matching of committed counter runs (no GPU needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_model():
    st = {"levels": 3, "chunk_suffixes": 900, "scattered_suffixes": 1000 + 600, "level_suffixes": 1000 + 700,
          "regathered": 50, "window_fetches": 300}
    m = bench.algorithmic_bytes(st, n_reads=10, n_bases=1000, tile_len=2048)
    assert m["local"] == 13 * 900 + 16 * 300 + 8 * 10
    assert m["level_scatter"] == 12.375 * 1000 + 24 * 600  # level 1 from the reads, then moves
    assert m["level_hist"] == 8 * 700 + 12 * 50  # level 1 counts keys from the reads
    assert m["final_emit"] == 13 * 100  # suffixes not finished in chunks
    assert m["level_scan"] == 2 * 1024 * 1700 / 2048
    # a build that never leaves level 1 scatters nothing at the later levels
    one = bench.algorithmic_bytes({"levels": 0, "chunk_suffixes": 1000}, 10, 1000)
    assert one["level_scatter"] == 0 and one["level_hist"] == 0


def test_counter_runs_match_sources_and_instantiation(tmp_path, monkeypatch):
    """Traffic per build from a counter record: raw FETCH_SIZE / WRITE_SIZE totals
    over the record's builds, scaled by its calibration factors."""
    (tmp_path / "profiles").mkdir()
    cal = {"fetch_factor": 2.0, "write_factor": 1.0, "note": "neg over 1 GiB"}

    def run(tuning, local_fetch, scatter):
        return {"tuning": tuning, "kernels": {
            "k_local": {"dispatches": 10, "fetch_MB": local_fetch, "write_MB": 20.0},
            "k_level_scatter": {"dispatches": 12, "fetch_MB": scatter, "write_MB": scatter},
            "k_gen_scatter": {"dispatches": 2, "fetch_MB": 6.0, "write_MB": 48.0}}}

    rec = {"kernel_sources_sha256_16": "abc", "builds": 2, "calibration": cal,
           "runs": [run("8x3", 100.0, 40.0), run("6x3", 200.0, 60.0)]}
    (tmp_path / "profiles" / "plain1_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "abc")
    # the chunk kernel's work depends on the chunk size only
    assert bench.measured_traffic("plain1", "local", "8x3") == (100 * 2 + 20) * 1e6 / 2
    assert bench.measured_traffic("plain1", "local", "16x3") == (100 * 2 + 20) * 1e6 / 2  # first run with chunk 3
    assert bench.measured_traffic("plain1", "local", "6x3") == (200 * 2 + 20) * 1e6 / 2  # its own run first
    assert bench.measured_traffic("plain1", "local", "8x6") is None
    # the scatters depend on both parts
    assert bench.measured_traffic("plain1", "level_scatter", "8x3") == (40 * 3 + 6 * 2 + 48) * 1e6 / 2
    assert bench.measured_traffic("plain1", "level_scatter", "6x3") == (60 * 3 + 6 * 2 + 48) * 1e6 / 2
    assert bench.measured_traffic("plain1", "level_scatter", "16x3") is None
    # other sources, or no counter run: nothing
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "other")
    assert bench.measured_traffic("plain1", "local", "8x3") is None
    assert bench.traffic_record("plain1") is None
    assert bench.measured_traffic("plain2", "local", "8x3") is None


def test_host_info_names_cpu_and_ram():
    info = bench.host_info()
    assert info["threads"] >= 1
    assert isinstance(info["cpu_model"], str) and info["cpu_model"]
    assert info["host_ram_gib"] is None or info["host_ram_gib"] > 0


def test_default_workload_is_the_largest_single_gpu_build():
    assert bench.DEFAULT_WORKLOAD == "plain2"
    assert bench.SECONDARY_WORKLOAD == "plain1"
    assert set(bench.CPU_SAMPLE_SCALE) == set(bench.WORKLOADS)
