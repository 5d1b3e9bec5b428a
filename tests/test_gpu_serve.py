"""Serving loop on the device: each job's result is the same alone and in the mix."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1401_7457_amd import cxbwt, datagen, serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    cxbwt.lib()


def test_served_jobs_match_alone_and_oracle():
    jobs = datagen.job_stream(count=12, rate_per_s=200.0, scale=0.002)
    print(f"[case] served: {len(jobs)} jobs, {sum(j.collection.n_bases for j in jobs)} bases", flush=True)
    sys.stdout.flush()
    ex = serve.DeviceExecutor()
    # a burst (every job arrives at once, staged in the loop): one batch holds them all
    rep, done = serve.replay([(0.0, j.collection) for j in jobs], ex, budget_bytes=8 << 30,
                             stage_in_background=False)
    assert rep["jobs_done"] == len(jobs)
    assert rep["batches"] == 1
    # the same jobs on their Poisson arrivals with the background stager
    rep2, done2 = serve.replay([(j.arrival_s, j.collection) for j in jobs], ex, budget_bytes=8 << 30)
    assert rep2["jobs_done"] == len(jobs)
    for a, b in zip(done, done2):
        assert np.array_equal(a.result[0], b.result[0]) and np.array_equal(a.result[1], b.result[1])
    for j in done:
        c = j.collection
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(j.result[0], eb) and np.array_equal(j.result[1], et)
        ab, at = cxbwt.build_host(c.text, c.offsets)
        assert np.array_equal(j.result[0], ab) and np.array_equal(j.result[1], at)


def test_served_batch_stays_within_admitted_footprints():
    """Device memory a served batch allocates (staged reads, batch copies,
    packed words, workspace, outputs) stays within the sum of the footprints
    the server admitted it with."""
    import torch
    jobs = datagen.job_stream(count=8, rate_per_s=1000.0, scale=0.004)
    ex = serve.DeviceExecutor(keep_on_device=True)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    print(f"[case] served footprint: {len(jobs)} jobs", flush=True)
    rep, done = serve.replay([(0.0, j.collection) for j in jobs], ex, budget_bytes=64 << 30,
                             stage_in_background=False)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    admitted = sum(j.footprint for j in done)
    assert rep["jobs_done"] == len(jobs) and rep["batches"] == 1
    assert peak <= admitted, f"peak {peak} bytes above the admitted {admitted}"
    for j in done:
        c = j.collection
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(j.result[0].cpu().numpy(), eb)
        assert np.array_equal(j.result[1].cpu().numpy().view(np.uint64), et)


def test_two_jobs_of_the_served_recipe_size():
    """Two jobs shaped like the served workload at full size (over 1M reads
    each, per-read lengths 100-250, own genomes at 1% error) served in one
    batch; each checked by the oracle's compiled checker and against its
    build alone."""
    rng = np.random.default_rng(4242)
    cols = []
    for n in (1_100_000, 1_300_000):
        genome = datagen.random_genome(rng, int(rng.integers(1_000_000, 10_000_001)))
        cols.append(datagen.sample_reads(rng, genome, n, rng.integers(100, 251, size=n), 0.01))
    print(f"[case] served recipe size: {[c.n_bases for c in cols]} bases", flush=True)
    ex = serve.DeviceExecutor()
    rep, done = serve.replay([(0.0, c) for c in cols], ex, budget_bytes=250 << 30, stage_in_background=False)
    assert rep["jobs_done"] == 2 and rep["batches"] == 1
    for j in done:
        c = j.collection
        assert oracle.check_bwt(j.result[0], j.result[1], c.text, c.offsets) == 0
        ab, at = cxbwt.build_host(c.text, c.offsets)
        assert np.array_equal(j.result[0], ab) and np.array_equal(j.result[1], at)
