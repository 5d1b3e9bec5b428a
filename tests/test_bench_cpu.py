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
    (tmp_path / "profiles").mkdir()
    rec = {"kernel_sources_sha256_16": "abc", "tuning": "8x3",
           "kernels": {"k_local": {"dispatches_per_build": 5, "fetch_MB_per_dispatch": 100.0,
                                   "write_MB_per_dispatch": 10.0},
                       "k_level_scatter": {"dispatches_per_build": 6, "fetch_MB_per_dispatch": 20.0,
                                           "write_MB_per_dispatch": 20.0},
                       "k_gen_scatter": {"dispatches_per_build": 1, "fetch_MB_per_dispatch": 6.0,
                                         "write_MB_per_dispatch": 48.0}}}
    (tmp_path / "profiles" / "plain1_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "abc")
    # the chunk kernel's work depends on the chunk size only
    assert bench.measured_traffic("plain1", "local", 5, "8x3") == 110e6
    assert bench.measured_traffic("plain1", "local", 5, "16x3") == 110e6
    assert bench.measured_traffic("plain1", "local", 5, "8x6") is None
    # the scatters depend on both parts
    assert bench.measured_traffic("plain1", "level_scatter", 7, "8x3") == (6 * 40e6 + 54e6) / 7
    assert bench.measured_traffic("plain1", "level_scatter", 7, "16x3") is None
    # counter runs of further instantiations of the same sources
    rec["other_tunings"] = [{"tuning": "6x3", "kernels": {
        "k_local": {"dispatches_per_build": 5, "fetch_MB_per_dispatch": 200.0, "write_MB_per_dispatch": 10.0},
        "k_level_scatter": {"dispatches_per_build": 6, "fetch_MB_per_dispatch": 30.0,
                            "write_MB_per_dispatch": 30.0}}}]
    (tmp_path / "profiles" / "plain1_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("plain1", "level_scatter", 6, "6x3") == 360e6 / 6
    assert bench.measured_traffic("plain1", "level_scatter", 7, "8x3") == (6 * 40e6 + 54e6) / 7
    assert bench.measured_traffic("plain1", "local", 5, "6x3") == 210e6  # its own run first
    assert bench.measured_traffic("plain1", "local", 5, "16x3") == 110e6
    assert bench.measured_traffic("plain1", "level_scatter", 7, "16x3") is None
    # other sources, or no counter run: nothing
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "other")
    assert bench.measured_traffic("plain1", "local", 5, "8x3") is None
    assert bench.measured_traffic("plain2", "local", 5, "8x3") is None
