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
