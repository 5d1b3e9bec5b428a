"""Every kernel instantiation the library holds gives the oracle's BWT, and
the autotuner selects one of them (device)."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1401_7457_amd import autotune, cxbwt, datagen

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    cxbwt.lib()
    before = cxbwt.get_tuning()
    yield
    cxbwt.set_tuning(*before)


def _inputs():
    rng = np.random.default_rng(31)
    out = [("plain0 x0.5", datagen.plain_config(0, scale=0.5)),
           ("2000x coverage", datagen.sample_reads(rng, datagen.random_genome(rng, 1500), 12000, 100, 0.001)),
           ("lengths 0..130", datagen.random_collection(rng, 3000, [0, 1, 26, 27, 28, 54, 81, 100, 130])),
           ("long reads", datagen.sample_reads(rng, datagen.random_genome(rng, 50_000), 600,
                                               rng.integers(150, 1500, size=600), 0.002))]
    return out


@pytest.mark.parametrize("choice", cxbwt.TUNING_CHOICES)
def test_every_instantiation_matches_oracle(choice):
    cxbwt.set_tuning(*choice)
    for label, col in _inputs():
        _say(f"tuning {choice}: {label} reads={col.n_reads} bases={col.n_bases}")
        b, t = cxbwt.build_host(col.text, col.offsets)
        eb, et = oracle.bwt(col.text, col.offsets)
        assert np.array_equal(b, eb), f"{choice} {label}: BWT differs"
        assert np.array_equal(t, et), f"{choice} {label}: term_pos differs"


@pytest.mark.parametrize("choice", cxbwt.TUNING_CHOICES)
def test_every_instantiation_batched(choice):
    cxbwt.set_tuning(*choice)
    rng = np.random.default_rng(32)
    cols = [datagen.random_collection(rng, int(rng.integers(1, 400)), [0, 5, 27, 60, 100]) for _ in range(12)]
    _say(f"tuning {choice}: batch of {len(cols)}")
    outs = cxbwt.build_batch_host(cols)
    for c, (b, t) in zip(cols, outs):
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(b, eb) and np.array_equal(t, et)


def test_autotuner_selects_a_choice_and_output_is_unchanged():
    import torch
    col = datagen.plain_config(0)
    _say(f"autotune plain0: reads={col.n_reads} bases={col.n_bases}")
    text = torch.from_numpy(col.text).cuda()
    off = torch.from_numpy(col.offsets.view(np.int64)).cuda()
    packed, _ = cxbwt.pack(text)
    res = autotune.tune_build(packed, off, col.n_reads, col.n_bases, col.max_read_len, repeats=3, persist=False)
    # every instantiation with the MSD schedule, and the stringword schedule
    assert set(res["ms"]) == set(autotune.choices_for(1))
    assert {ch[:2] for ch in res["ms"]} == set(cxbwt.TUNING_CHOICES)
    assert res["choice"] in res["ms"]
    assert autotune.current() == res["choice"]
    assert autotune.select_for(col.n_reads, col.n_bases, col.max_read_len) == res["choice"]
    try:
        b, t = cxbwt.build_host(col.text, col.offsets)
    finally:
        autotune.apply((*cxbwt.TUNING_CHOICES[0], cxbwt.SCHEDULE_MSD))
    eb, et = oracle.bwt(col.text, col.offsets)
    assert np.array_equal(b, eb) and np.array_equal(t, et)


def test_tuner_choice_persists_across_processes(tmp_path, monkeypatch):
    """A tuned choice is written to the cache file and found again by a fresh
    in-memory cache (a later process)."""
    import torch
    monkeypatch.setenv("CXBWT_TUNE_CACHE", str(tmp_path / "tuning.json"))
    col = datagen.plain_config(0, scale=0.2)
    text = torch.from_numpy(col.text).cuda()
    off = torch.from_numpy(col.offsets.view(np.int64)).cuda()
    packed, _ = cxbwt.pack(text)
    _say("autotune persistence")
    choices = ((8, 3, cxbwt.SCHEDULE_MSD), (16, 6, cxbwt.SCHEDULE_MSD))
    res = autotune.tune_build(packed, off, col.n_reads, col.n_bases, col.max_read_len, repeats=1, choices=choices)
    try:
        monkeypatch.setattr(autotune, "_cache", {})
        autotune.apply((*cxbwt.TUNING_CHOICES[0], cxbwt.SCHEDULE_MSD))
        assert autotune.select_for(col.n_reads, col.n_bases, col.max_read_len) == res["choice"]
        assert autotune.current() == res["choice"]
    finally:
        autotune.apply((*cxbwt.TUNING_CHOICES[0], cxbwt.SCHEDULE_MSD))
