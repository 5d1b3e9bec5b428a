"""Serving loop: BWT-build jobs admitted under an HBM budget, continuously batched.

Jobs (read collections) arrive over time.  The scheduler:
  * rejects a job whose footprint exceeds the whole budget;
  * admits queued jobs in arrival order while the resident footprint stays
    within the budget (an admitted job's reads are staged on the device by a
    background stager thread, overlapping the build that is running);
  * whenever fewer than `max_inflight` batches are building, starts every
    staged job that fits the batch limits as ONE batched build that returns
    at once (cxbwt_build_batch_start, on a stream of its own): continuous
    batching, with the next batch's staging, packing and level launches
    overlapping the running one on the device;
  * collects finished batches, returns results per job, frees their memory
    and admits more.
A batch that fails is retried job by job so that a bad job fails alone.

The executor is an interface: DeviceExecutor drives the HIP library; tests
plug in a CPU executor.  The clock is injectable for deterministic tests.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

QUEUED, ADMITTED, STAGED, RUNNING, DONE, FAILED, CANCELLED = (
    "queued", "admitted", "staged", "running", "done", "failed", "cancelled")


@dataclass
class Job:
    id: int
    collection: object
    arrival_s: float
    footprint: int = 0
    state: str = QUEUED
    result: Optional[tuple] = None
    error: Optional[str] = None
    t_admit: Optional[float] = None
    t_start: Optional[float] = None
    t_done: Optional[float] = None
    handle: object = None  # executor-owned staging state
    batch_id: Optional[int] = None
    done_event: threading.Event = field(default_factory=threading.Event)

    @property
    def latency_s(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival_s

    def wait(self, timeout=None):
        self.done_event.wait(timeout)
        return self.result


class Executor:
    """What the scheduler needs from a device."""

    def footprint(self, col) -> int:  # pragma: no cover - interface
        raise NotImplementedError

    def stage(self, job: Job) -> None:  # pragma: no cover - interface
        raise NotImplementedError

    def run_batch(self, jobs: list[Job]) -> list[tuple]:  # pragma: no cover - interface
        raise NotImplementedError

    def release(self, job: Job) -> None:  # pragma: no cover - interface
        raise NotImplementedError

    # Batches that return at once.  The defaults build synchronously.
    def start_batch(self, jobs: list[Job]):
        try:
            return (self.run_batch(jobs), None)
        except Exception as e:  # reported by finish_batch
            return (None, e)

    def batch_done(self, handle) -> bool:
        return True

    def finish_batch(self, handle) -> list[tuple]:
        results, err = handle
        if err is not None:
            raise err
        return results


def state_bytes(n_reads: int, n_bases: int, max_read_len: int = 255) -> int:
    """Device bytes a job holds while resident and while its batch runs.

    Staged ASCII reads (B) + its part of the batch's concatenated reads (B),
    packed words (B/4 + 16), offsets (8n + 8), outputs (B + n bytes of BWT,
    8n of term_pos), and the library's workspace for the job alone
    (cxbwt_batch_workspace_bytes for one collection, pure host arithmetic;
    a batch's workspace is at most the sum of its jobs').  0 reads or bases
    beyond one build's limit: the job cannot be built (None).
    """
    from . import cxbwt
    ws = cxbwt.batch_workspace_bytes(max(1, n_reads), n_bases, max(1, min(max_read_len, 65535)), 1)
    if ws == 0:
        return None
    return int(ws + 2 * n_bases + n_bases // 4 + 16 + 8 * (n_reads + 1) + n_bases + n_reads + 8 * n_reads + 4096)


def footprint_of(col) -> Optional[int]:
    return state_bytes(col.n_reads, col.n_bases, col.max_read_len)


class DeviceExecutor(Executor):
    """Stages jobs on the device and builds batches with cxbwt_build_batch.

    keep_on_device: results stay as device tensors (latency = device
    completion, the copy to the host is the caller's); otherwise they are
    copied to host arrays before the job completes.
    """

    def __init__(self, device="cuda", keep_on_device: bool = False):
        import torch

        from . import cxbwt
        self.torch = torch
        self.cx = cxbwt
        self.device = torch.device(device)
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.keep_on_device = keep_on_device
        self.build_streams = [torch.cuda.Stream(device=self.device) for _ in range(2)]
        self._next_stream = 0
        cxbwt.lib()

    def footprint(self, col) -> Optional[int]:
        return footprint_of(col)

    def stage(self, job: Job) -> None:
        """Copy the job's reads to the device on the copy stream.  The reads may
        be a numpy array or a torch CPU tensor; a client that receives reads
        into pinned host memory (a tensor with pin_memory) gets an
        asynchronous copy at full link speed."""
        torch = self.torch
        col = job.collection
        src = col.text if isinstance(col.text, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(col.text))
        with torch.cuda.stream(self.copy_stream):
            t_dev = src.to(self.device, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy_stream)
        job.handle = (t_dev, ev)

    def run_batch(self, jobs: list[Job]) -> list[tuple]:
        return self.finish_batch(self.start_batch(jobs))

    def start_batch(self, jobs: list[Job]):
        """Concatenate the staged reads, pack them and start the batched build
        on the next of two build streams; returns at once."""
        from . import autotune
        torch, cx = self.torch, self.cx
        stream = self.build_streams[self._next_stream % len(self.build_streams)]
        self._next_stream += 1
        cols = [j.collection for j in jobs]
        _, offsets_h, coll_reads, maxlen = cx.concat_collections([_Shape(c) for c in cols])
        nbs = [c.n_bases for c in cols]
        ns = [c.n_reads for c in cols]
        n, nb = int(coll_reads[-1]), int(offsets_h[-1])
        with torch.cuda.stream(stream):
            for j in jobs:
                stream.wait_event(j.handle[1])
                j.handle[0].record_stream(stream)  # staged on the copy stream, read on this one
            texts = [j.handle[0] for j in jobs]
            text = torch.cat(texts) if nb else torch.empty(0, dtype=torch.uint8, device=self.device)
            offsets = torch.from_numpy(offsets_h.view(np.int64)).to(self.device, non_blocking=False)
            packed, pstatus = cx.pack(text, stream=stream)
            # the autotuner's remembered choice for this shape class, if it has
            # one, as this build's own options (the thread's choices otherwise)
            opts = autotune.remembered(n, nb, maxlen, len(jobs))
            job = cx.build_batch_start(packed, offsets, n, nb, maxlen, coll_reads, stream=stream, opts=opts)
        return (job, pstatus, ns, nbs)

    def batch_done(self, handle) -> bool:
        return handle[0].done()

    def finish_batch(self, handle) -> list[tuple]:
        job, pstatus, ns, nbs = handle
        bwt, term = job.wait()
        if int(pstatus.item()) != 0:
            raise self.cx.CxbwtError(self.cx.EDATA, "cxbwt_pack (non-ACGT byte)")
        if not self.keep_on_device:
            bwt = bwt.cpu().numpy()
            term = term.cpu().numpy().view(np.uint64)
        out, b0, r0 = [], 0, 0
        for nj, nbj in zip(ns, nbs):
            out.append((bwt[b0:b0 + nj + nbj], term[r0:r0 + nj]))
            b0 += nj + nbj
            r0 += nj
        return out

    def release(self, job: Job) -> None:
        job.handle = None


class _Failed:
    """A batch whose start raised: finished, failed, isolated job by job."""

    def __init__(self, error):
        self.error = error


class _Shape:
    """Offsets-only view of a collection (the batch's text is already on the device)."""

    def __init__(self, col):
        self.offsets = col.offsets
        self.text = np.zeros(0, dtype=np.uint8)


class Server:
    """Continuous-batching BWT build server over an Executor.

    budget_bytes      device memory the resident jobs may hold together
    max_batch_bases   bases per batch (the device path takes < 2^32)
    max_batch_jobs    jobs per batch (1 with max_inflight 1 = one job at a time, the baseline)
    max_inflight      batches building at once (each on a stream of its own)
    """

    def __init__(self, executor: Executor, budget_bytes: int, max_batch_bases: int = (1 << 32) - 1,
                 max_batch_jobs: Optional[int] = None, clock: Callable[[], float] = time.monotonic,
                 stage_in_background: bool = True, max_inflight: int = 2):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_batch_bases = int(max_batch_bases)
        self.max_batch_jobs = max_batch_jobs
        self.max_inflight = max(1, int(max_inflight))
        self.inflight: list = []               # (batch, executor handle)
        self.clock = clock
        self.queue: deque[Job] = deque()       # arrived, not admitted
        self.staged: deque[Job] = deque()      # resident, waiting for a batch
        self.resident = 0
        self.jobs: list[Job] = []
        self.batches: list[list[int]] = []
        self._next_id = 0
        self._lock = threading.Lock()
        self._stage_q: deque[Job] = deque()
        self._stage_cv = threading.Condition(self._lock)
        self._stop = False
        self._stager = None
        if stage_in_background:
            self._stager = threading.Thread(target=self._stage_loop, daemon=True)
            self._stager.start()

    # ---- submission ---------------------------------------------------------
    def submit(self, collection, arrival_s: Optional[float] = None) -> Job:
        with self._lock:
            job = Job(self._next_id, collection, self.clock() if arrival_s is None else arrival_s)
            self._next_id += 1
            job.footprint = self.ex.footprint(collection)
            self.jobs.append(job)
            if job.footprint is None:
                job.footprint = 0
                self._finish(job, FAILED, error="collection above the size one build takes")
            elif job.footprint > self.budget:
                self._finish(job, FAILED, error="footprint exceeds the whole device budget")
            else:
                self.queue.append(job)
            return job

    def cancel(self, job: Job) -> bool:
        with self._lock:
            if job.state in (QUEUED,):
                self.queue.remove(job)
            elif job.state in (ADMITTED, STAGED):
                if job in self.staged:
                    self.staged.remove(job)
                if job in self._stage_q:
                    self._stage_q.remove(job)
                self.resident -= job.footprint
                self.ex.release(job)
            else:
                return False
            self._finish(job, CANCELLED)
            return True

    # ---- scheduling ---------------------------------------------------------
    def _finish(self, job: Job, state: str, result=None, error=None):
        job.state = state
        job.result = result
        job.error = error
        job.t_done = self.clock()
        job.done_event.set()

    def _admit(self):
        """Admit queued jobs (arrival order) while the budget allows."""
        now = self.clock()
        while self.queue and self.queue[0].arrival_s <= now:
            job = self.queue[0]
            if self.resident + job.footprint > self.budget:
                break  # waits for memory: FIFO, no overtaking
            self.queue.popleft()
            self.resident += job.footprint
            job.state = ADMITTED
            job.t_admit = now
            if self._stager is not None:
                self._stage_q.append(job)
                self._stage_cv.notify()
            else:
                self._stage_now(job)

    def _stage_now(self, job: Job):
        try:
            self.ex.stage(job)
        except Exception as e:  # staging failure fails only this job
            self.resident -= job.footprint
            self._finish(job, FAILED, error=f"staging: {e}")
            return
        if job.state == ADMITTED:
            job.state = STAGED
            self.staged.append(job)

    def _stage_loop(self):
        while True:
            with self._lock:
                while not self._stage_q and not self._stop:
                    self._stage_cv.wait()
                if self._stop:
                    return
                job = self._stage_q.popleft()
            try:
                self.ex.stage(job)
                ok, err = True, None
            except Exception as e:
                ok, err = False, e
            with self._lock:
                if job.state != ADMITTED:
                    self.ex.release(job)  # cancelled meanwhile
                    continue
                if ok:
                    job.state = STAGED
                    self.staged.append(job)
                else:
                    self.resident -= job.footprint
                    self._finish(job, FAILED, error=f"staging: {err}")
                self._stage_cv.notify_all()

    def _take_batch(self) -> list[Job]:
        batch, bases = [], 0
        while self.staged:
            j = self.staged[0]
            nb = j.collection.n_bases
            if batch and (bases + nb > self.max_batch_bases or
                          (self.max_batch_jobs and len(batch) >= self.max_batch_jobs)):
                break
            self.staged.popleft()
            batch.append(j)
            bases += nb
        return batch

    def step(self) -> int:
        """Collect finished batches, admit what fits, and start batches of
        staged jobs while fewer than max_inflight are building.  Returns the
        jobs finished or started (0: nothing to do yet)."""
        progress = self._reap()
        while len(self.inflight) < self.max_inflight:
            with self._lock:
                self._admit()
                batch = self._take_batch()
                for j in batch:
                    j.state = RUNNING
                    j.t_start = self.clock()
                    j.batch_id = len(self.batches)
                if batch:
                    self.batches.append([j.id for j in batch])
            if not batch:
                break
            try:
                handle = self.ex.start_batch(batch)
            except Exception as e:
                handle = _Failed(e)  # finished (failed) at once: isolated when reaped
            self.inflight.append((batch, handle))
            progress += len(batch)
            progress += self._reap()  # an executor that builds synchronously finishes at once
        return progress

    def _reap(self) -> int:
        """Finish the in-flight batches whose builds are done."""
        done = 0
        for batch, handle in list(self.inflight):
            if not isinstance(handle, _Failed) and not self.ex.batch_done(handle):
                continue
            self.inflight.remove((batch, handle))
            self._complete(batch, handle)
            done += len(batch)
        return done

    def _complete(self, batch, handle):
        try:
            if isinstance(handle, _Failed):
                raise handle.error
            results = self.ex.finish_batch(handle)
            failures = {}
        except Exception:
            # isolate: rebuild one by one so only the bad job fails
            results, failures = [], {}
            for j in batch:
                try:
                    results.append(self.ex.run_batch([j])[0])
                except Exception as e:
                    results.append(None)
                    failures[j.id] = str(e)
        with self._lock:
            for j, r in zip(batch, results):
                self.resident -= j.footprint
                self.ex.release(j)
                if j.state == CANCELLED:
                    continue
                if j.id in failures:
                    self._finish(j, FAILED, error=failures[j.id])
                else:
                    self._finish(j, DONE, result=r)

    def pending(self) -> int:
        with self._lock:
            return sum(1 for j in self.jobs if j.state in (QUEUED, ADMITTED, STAGED, RUNNING))

    def run_until_idle(self, sleep: Callable[[float], None] = time.sleep, poll_s: float = 0.0005,
                       max_wall_s: Optional[float] = None):
        """Drive the loop until every submitted job is finished."""
        t0 = time.monotonic()
        while self.pending():
            built = self.step()
            if built:
                continue
            if max_wall_s is not None and time.monotonic() - t0 > max_wall_s:
                raise TimeoutError("server did not drain in time")
            with self._lock:
                nxt = self.queue[0].arrival_s if self.queue else None
                waiting_stage = bool(self._stage_q) or any(j.state == ADMITTED for j in self.jobs)
            now = self.clock()
            if nxt is not None and nxt > now and not waiting_stage and not self.staged:
                sleep(min(nxt - now, 0.05))
            else:
                sleep(poll_s)

    def close(self):
        with self._lock:
            self._stop = True
            self._stage_cv.notify_all()
        if self._stager is not None:
            self._stager.join(timeout=5)

    # ---- reporting ------------------------------------------------------------
    def report(self) -> dict:
        done = [j for j in self.jobs if j.state == DONE]
        if not done:
            return {"jobs_done": 0}
        lat = np.array([j.latency_s for j in done])
        first = min(j.arrival_s for j in done)
        last = max(j.t_done for j in done)
        bases = sum(j.collection.n_bases for j in done)
        return {
            "jobs_done": len(done),
            "jobs_failed": sum(1 for j in self.jobs if j.state == FAILED),
            "bases": bases,
            "makespan_s": last - first,
            "gbases_per_s": bases / max(last - first, 1e-12) / 1e9,
            "latency_p50_s": float(np.percentile(lat, 50)),
            "latency_p99_s": float(np.percentile(lat, 99)),
            "batches": len(self.batches),
            "mean_jobs_per_batch": float(np.mean([len(b) for b in self.batches])) if self.batches else 0.0,
        }


def replay(arrivals, executor: Executor, budget_bytes: int, **server_kw):
    """Run a trace in real time: [(arrival_s, collection), ...] relative to now.

    Returns (report dict, list of jobs in submission order).
    """
    srv = Server(executor, budget_bytes, **server_kw)
    try:
        t0 = srv.clock()
        jobs = [srv.submit(col, arrival_s=t0 + a) for a, col in arrivals]
        srv.run_until_idle()
        return srv.report(), jobs
    finally:
        srv.close()


def plan_waves(sizes: list[tuple], max_bases: int = (1 << 32) - 1, budget_bytes: Optional[int] = None):
    """Group collections (n_reads, n_bases[, max_read_len]) into consecutive waves for batched builds.

    Each wave holds fewer than max_bases bases in total and, if budget_bytes is
    given, a footprint within it.  Returns lists of collection indices.
    """
    waves, cur, bases, foot = [], [], 0, 0
    for i, size in enumerate(sizes):
        n, nb = size[0], size[1]
        f = state_bytes(n, nb, size[2] if len(size) > 2 else 255) or 0
        if cur and (bases + nb > max_bases or (budget_bytes is not None and foot + f > budget_bytes)):
            waves.append(cur)
            cur, bases, foot = [], 0, 0
        cur.append(i)
        bases += nb
        foot += f
    if cur:
        waves.append(cur)
    return waves
