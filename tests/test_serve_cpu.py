"""Serving scheduler on the CPU: a fake executor behind the same interface.

The fake executor computes each job's BWT with the oracle and advances a
virtual clock by a simulated build time, so admission, batching, failure
isolation, cancellation and latency bookkeeping are checked exactly.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1401_7457_amd import datagen, serve


class VClock:
    def __init__(self):
        self.now = 0.0

    def __call__(self):
        return self.now

    def sleep(self, dt):
        self.now += max(dt, 1e-6)


class FakeExecutor(serve.Executor):
    def __init__(self, clock, per_base_s=1e-6, fixed_s=0.01, fail_ids=(), budget_probe=None):
        self.clock = clock
        self.per_base_s = per_base_s
        self.fixed_s = fixed_s
        self.fail_ids = set(fail_ids)
        self.batches = []
        self.staged = set()
        self.budget_probe = budget_probe

    def footprint(self, col):
        return serve.state_bytes(col.n_reads, col.n_bases)

    def stage(self, job):
        job.handle = ("staged", job.id)
        self.staged.add(job.id)

    def run_batch(self, jobs):
        if self.budget_probe:
            self.budget_probe()
        self.batches.append([j.id for j in jobs])
        if any(j.id in self.fail_ids for j in jobs):
            raise RuntimeError("injected device failure")
        self.clock.now += self.fixed_s + self.per_base_s * sum(j.collection.n_bases for j in jobs)
        return [oracle.bwt(j.collection.text, j.collection.offsets) for j in jobs]

    def release(self, job):
        self.staged.discard(job.id)
        job.handle = None


def _cols(k, n=30, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        g = datagen.random_genome(rng, 2000)
        out.append(datagen.sample_reads(rng, g, int(rng.integers(5, n)), 50, 0.01))
    return out


def _server(ex, clock, budget=10 ** 9, **kw):
    return serve.Server(ex, budget, clock=clock, stage_in_background=False, **kw)


def test_all_jobs_complete_with_oracle_results():
    vc = VClock()
    ex = FakeExecutor(vc)
    srv = _server(ex, vc)
    cols = _cols(8)
    jobs = [srv.submit(c, arrival_s=0.001 * i) for i, c in enumerate(cols)]
    srv.run_until_idle(sleep=vc.sleep)
    for j, c in zip(jobs, cols):
        assert j.state == serve.DONE
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(j.result[0], eb) and np.array_equal(j.result[1], et)
    assert ex.staged == set()  # everything released


def test_continuous_batching_joins_arrivals_during_a_build():
    vc = VClock()
    ex = FakeExecutor(vc, per_base_s=0.0, fixed_s=1.0)
    srv = _server(ex, vc)
    cols = _cols(6)
    srv.submit(cols[0], arrival_s=0.0)
    # these arrive while the first batch (1 s) is running
    for i in range(1, 6):
        srv.submit(cols[i], arrival_s=0.1 * i)
    srv.run_until_idle(sleep=vc.sleep)
    assert ex.batches == [[0], [1, 2, 3, 4, 5]]
    assert srv.report()["batches"] == 2


def test_one_job_at_a_time_baseline():
    vc = VClock()
    ex = FakeExecutor(vc, per_base_s=0.0, fixed_s=1.0)
    srv = _server(ex, vc, max_batch_jobs=1)
    for i, c in enumerate(_cols(4)):
        srv.submit(c, arrival_s=0.0)
    srv.run_until_idle(sleep=vc.sleep)
    assert ex.batches == [[0], [1], [2], [3]]


def test_budget_makes_jobs_wait_and_is_never_exceeded():
    vc = VClock()
    cols = _cols(6, n=40)
    fp = [serve.state_bytes(c.n_reads, c.n_bases) for c in cols]
    budget = max(fp) * 2
    holder = {}

    def probe():
        assert holder["srv"].resident <= budget

    ex = FakeExecutor(vc, per_base_s=0.0, fixed_s=1.0, budget_probe=probe)
    srv = _server(ex, vc, budget=budget)
    holder["srv"] = srv
    for c in cols:
        srv.submit(c, arrival_s=0.0)
    srv.run_until_idle(sleep=vc.sleep)
    assert all(j.state == serve.DONE for j in srv.jobs)
    assert sum(fp) > budget  # not everything fits at once, so some jobs waited
    for b in ex.batches:
        assert sum(fp[i] for i in b) <= budget
    assert len(ex.batches) >= 2


def test_job_larger_than_the_budget_is_rejected():
    vc = VClock()
    ex = FakeExecutor(vc)
    srv = _server(ex, vc, budget=1000)
    j = srv.submit(_cols(1)[0], arrival_s=0.0)
    assert j.state == serve.FAILED and "budget" in j.error
    srv.run_until_idle(sleep=vc.sleep)
    assert ex.batches == []


def test_failure_of_one_job_fails_only_that_job():
    vc = VClock()
    ex = FakeExecutor(vc, fail_ids={2})
    srv = _server(ex, vc)
    cols = _cols(5)
    jobs = [srv.submit(c, arrival_s=0.0) for c in cols]
    srv.run_until_idle(sleep=vc.sleep)
    assert [j.state for j in jobs] == [serve.DONE, serve.DONE, serve.FAILED, serve.DONE, serve.DONE]
    assert "injected" in jobs[2].error
    for j, c in zip(jobs, cols):
        if j.state == serve.DONE:
            assert np.array_equal(j.result[0], oracle.bwt(c.text, c.offsets)[0])


def test_cancel_queued_job():
    vc = VClock()
    ex = FakeExecutor(vc)
    srv = _server(ex, vc)
    cols = _cols(3)
    a = srv.submit(cols[0], arrival_s=0.0)
    b = srv.submit(cols[1], arrival_s=5.0)
    assert srv.cancel(b)
    srv.run_until_idle(sleep=vc.sleep)
    assert a.state == serve.DONE and b.state == serve.CANCELLED
    assert all(1 not in batch for batch in ex.batches)


def test_latency_bookkeeping_on_a_virtual_clock():
    vc = VClock()
    ex = FakeExecutor(vc, per_base_s=0.0, fixed_s=2.0)
    srv = _server(ex, vc, max_batch_jobs=1)
    cols = _cols(3)
    jobs = [srv.submit(c, arrival_s=0.0) for c in cols]
    srv.run_until_idle(sleep=vc.sleep)
    # FIFO, one at a time, 2 s each: done at 2, 4, 6
    assert [pytest.approx(j.latency_s) for j in jobs] == [2.0, 4.0, 6.0]
    rep = srv.report()
    assert rep["latency_p50_s"] == pytest.approx(4.0)
    assert rep["jobs_done"] == 3


def test_background_stager_thread_path():
    vc = VClock()
    ex = FakeExecutor(vc)
    srv = serve.Server(ex, 10 ** 9, clock=vc, stage_in_background=True)
    try:
        cols = _cols(4)
        jobs = [srv.submit(c, arrival_s=0.0) for c in cols]
        srv.run_until_idle(sleep=lambda dt: (vc.sleep(dt), __import__("time").sleep(0.001)), max_wall_s=30)
        assert all(j.state == serve.DONE for j in jobs)
    finally:
        srv.close()


def test_plan_waves_respects_limits():
    sizes = [(10, 1000), (10, 3000), (10, 500), (10, 4000), (10, 100)]
    waves = serve.plan_waves(sizes, max_bases=4500)
    assert waves == [[0, 1, 2], [3, 4]]
    assert all(sum(sizes[i][1] for i in w) <= 4500 for w in waves)
    assert sorted(i for w in waves for i in w) == list(range(5))


class AsyncFakeExecutor(FakeExecutor):
    """Batches that return at once and finish after their simulated build time
    on the virtual clock; records how many were building together."""

    def __init__(self, clock, **kw):
        super().__init__(clock, **kw)
        self.running = []
        self.max_running = 0

    def start_batch(self, jobs):
        self.batches.append([j.id for j in jobs])
        res = [oracle.bwt(j.collection.text, j.collection.offsets) for j in jobs]
        end = self.clock.now + self.fixed_s + self.per_base_s * sum(j.collection.n_bases for j in jobs)
        h = {"end": end, "res": res}
        self.running.append(h)
        self.max_running = max(self.max_running, len(self.running))
        return h

    def batch_done(self, h):
        return self.clock.now >= h["end"]

    def finish_batch(self, h):
        self.running.remove(h)
        return h["res"]


def test_batches_overlap_up_to_max_inflight():
    clk = VClock()
    ex = AsyncFakeExecutor(clk, per_base_s=1e-6, fixed_s=0.01)
    srv = serve.Server(ex, budget_bytes=1 << 40, max_batch_jobs=2, clock=clk, stage_in_background=False,
                       max_inflight=2)
    cols = _cols(8, seed=5)
    jobs = [srv.submit(c, arrival_s=0.0) for c in cols]
    srv.run_until_idle(sleep=clk.sleep)
    assert ex.max_running == 2
    for j, c in zip(jobs, cols):
        assert j.state == serve.DONE
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(j.result[0], eb) and np.array_equal(j.result[1], et)
    # one at a time: never two building together
    clk2 = VClock()
    ex2 = AsyncFakeExecutor(clk2, per_base_s=1e-6, fixed_s=0.01)
    srv2 = serve.Server(ex2, budget_bytes=1 << 40, max_batch_jobs=1, clock=clk2, stage_in_background=False,
                        max_inflight=1)
    for c in cols:
        srv2.submit(c, arrival_s=0.0)
    srv2.run_until_idle(sleep=clk2.sleep)
    assert ex2.max_running == 1
    assert srv2.report()["makespan_s"] > srv.report()["makespan_s"]
