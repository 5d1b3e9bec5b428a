"""Builds that return at once (cxbwt_build_start / cxbwt_build_batch_start):
two builds started back to back on two streams, and batches, each compared
with the oracle; a failing started build reports its status at the wait."""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1401_7457_amd import cxbwt, datagen

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


def _device(col, stream):
    import torch
    with torch.cuda.stream(stream):
        text = torch.from_numpy(col.text).cuda() if col.n_bases else torch.empty(0, dtype=torch.uint8,
                                                                                   device="cuda")
        offs = torch.from_numpy(col.offsets.view(np.int64)).cuda()
        packed, status = cxbwt.pack(text, stream=stream)
    return text, offs, packed, status


def _against_oracle(col, bwt, term, label):
    eb, et = oracle.bwt(col.text, col.offsets)
    b = bwt.cpu().numpy()
    assert np.array_equal(b, eb), f"{label}: {np.count_nonzero(b != eb)} BWT rows differ"
    assert np.array_equal(term.cpu().numpy().view(np.uint64), et), f"{label}: term_pos differs"


def test_two_builds_on_two_streams_back_to_back():
    import torch
    cols = [datagen.plain_config(0), datagen.plain_config(2, scale=0.002)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    _say(f"two streams: {[c.n_bases for c in cols]} bases")
    inputs = [_device(c, s) for c, s in zip(cols, streams)]
    jobs = []
    for c, s, (text, offs, packed, status) in zip(cols, streams, inputs):
        jobs.append(cxbwt.build_start(packed, offs, c.n_reads, c.n_bases, c.max_read_len, stream=s))
    # both calls have returned; the builds run (and may overlap) on the device
    outs = [j.wait() for j in jobs]
    for c, s, (b, t), (_, _, _, status), j in zip(cols, streams, outs, inputs, jobs):
        s.synchronize()
        assert int(status.item()) == 0
        assert j.stats["levels"] >= 1
        _against_oracle(c, b, t, c.label)


def test_started_builds_match_blocking_builds_many_in_flight():
    """Six builds on three streams, all started before any is waited for."""
    import torch
    rng = np.random.default_rng(9)
    cols = [datagen.random_collection(rng, int(rng.integers(50, 3000)), [0, 1, 27, 54, 100, 150])
            for _ in range(6)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    _say(f"six builds on three streams: {[c.n_bases for c in cols]} bases")
    jobs = []
    for i, c in enumerate(cols):
        s = streams[i % 3]
        _, offs, packed, _ = _device(c, s)
        jobs.append((c, cxbwt.build_start(packed, offs, c.n_reads, c.n_bases, c.max_read_len, stream=s)))
    for c, j in jobs:
        b, t = j.wait()
        _against_oracle(c, b, t, "in flight")


def test_started_batch_and_polling():
    import torch
    cols = datagen.batch_collections(count=10, scale=0.005)
    text, offsets, coll_reads, maxlen = cxbwt.concat_collections(cols)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        t_dev = torch.from_numpy(text).cuda()
        o_dev = torch.from_numpy(offsets.view(np.int64)).cuda()
        packed, _ = cxbwt.pack(t_dev, stream=s)
    n, nb = offsets.size - 1, int(offsets[-1])
    _say(f"started batch: {len(cols)} collections, {nb} bases")
    job = cxbwt.build_batch_start(packed, o_dev, n, nb, maxlen, coll_reads, stream=s)
    import time
    t0 = time.monotonic()
    while not job.done() and time.monotonic() - t0 < 60:
        time.sleep(0.0005)
    assert job.done()
    bwt, term = job.wait()
    outs = cxbwt.split_batch_output(bwt.cpu().numpy(), term.cpu().numpy().view(np.uint64), cols)
    for c, (b, t) in zip(cols, outs):
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(b, eb) and np.array_equal(t, et)


def test_started_build_reports_bad_offsets_at_the_wait():
    import torch
    col = datagen.plain_config(0, scale=0.05)
    s = torch.cuda.Stream()
    _, offs, packed, _ = _device(col, s)
    with torch.cuda.stream(s):
        bad = offs.clone()
        bad[5] = bad[7] + 3  # offsets decrease: found by the device
    _say("started build with invalid offsets")
    job = cxbwt.build_start(packed, bad, col.n_reads, col.n_bases, col.max_read_len, stream=s)
    with pytest.raises(cxbwt.CxbwtError) as e:
        job.wait()
    assert e.value.status == cxbwt.EDATA
    # the stream and the library stay usable
    job = cxbwt.build_start(packed, offs, col.n_reads, col.n_bases, col.max_read_len, stream=s)
    b, t = job.wait()
    _against_oracle(col, b, t, "after the failure")


def test_started_builds_with_their_own_options():
    """Per-call options: the same input built with every instantiation and
    both schedules, all started before any wait, each on its own stream; the
    thread's own choices are left alone."""
    import torch
    col = datagen.plain_config(0, scale=0.2)
    before = (cxbwt.get_tuning(), cxbwt.get_schedule())
    choices = [(t, c, cxbwt.SCHEDULE_MSD, 1) for t, c in cxbwt.TUNING_CHOICES[:3]]
    choices.append((*cxbwt.TUNING_CHOICES[0], cxbwt.SCHEDULE_STRINGWORD, 1))
    _say(f"started builds with options {choices}: {col.n_bases} bases")
    streams = [torch.cuda.Stream() for _ in choices]
    jobs = []
    for ch, s in zip(choices, streams):
        _, offs, packed, _ = _device(col, s)
        jobs.append((ch, cxbwt.build_start(packed, offs, col.n_reads, col.n_bases, col.max_read_len, stream=s,
                                           opts=ch)))
    for ch, j in jobs:
        b, t = j.wait()
        assert j.stats["schedule"] == ch[2]
        assert sum(j.stats["ms"].values()) > 0  # timing was asked for
        _against_oracle(col, b, t, f"options {ch}")
    assert (cxbwt.get_tuning(), cxbwt.get_schedule()) == before


def test_device_failure_text():
    """An EDATA from the device comes with the library's text."""
    import torch
    col = datagen.plain_config(0, scale=0.05)
    s = torch.cuda.Stream()
    _, offs, packed, _ = _device(col, s)
    with torch.cuda.stream(s):
        bad = offs.clone()
        bad[3] = bad[9] + 1
    _say("blocking build with invalid offsets: error text")
    with pytest.raises(cxbwt.CxbwtError) as e:
        with torch.cuda.stream(s):
            cxbwt.build(packed, bad, col.n_reads, col.n_bases, col.max_read_len, stream=s)
    assert e.value.status == cxbwt.EDATA
    assert e.value.detail, "no text for EDATA"


def test_blocking_builds_take_options():
    """cxbwt_build / cxbwt_build_batch with their own options: the result is the
    oracle's for every choice, the statistics name the schedule run, and the
    thread's own choices are left as they were."""
    import torch
    col = datagen.plain_config(0, scale=0.1)
    before = (cxbwt.get_tuning(), cxbwt.get_schedule())
    s = torch.cuda.current_stream()
    _, offs, packed, _ = _device(col, s)
    for ch in ((*cxbwt.TUNING_CHOICES[-1], cxbwt.SCHEDULE_MSD, 1), (*cxbwt.TUNING_CHOICES[0], cxbwt.SCHEDULE_STRINGWORD, 0)):
        _say(f"blocking build with options {ch}")
        b, t = cxbwt.build(packed, offs, col.n_reads, col.n_bases, col.max_read_len, opts=ch)
        assert cxbwt.last_stats()["schedule"] == ch[2]
        _against_oracle(col, b, t, f"options {ch}")
    cols = datagen.batch_collections(count=5, scale=0.002)
    text, offsets, coll_reads, maxlen = cxbwt.concat_collections(cols)
    t_dev = torch.from_numpy(text).cuda()
    o_dev = torch.from_numpy(offsets.view(np.int64)).cuda()
    packed_b, _ = cxbwt.pack(t_dev)
    n, nb = offsets.size - 1, int(offsets[-1])
    _say(f"blocking batch with options: {len(cols)} collections, {nb} bases")
    bwt, term = cxbwt.build_batch(packed_b, o_dev, n, nb, maxlen, coll_reads,
                                  opts=(*cxbwt.TUNING_CHOICES[-1], cxbwt.SCHEDULE_MSD))
    outs = cxbwt.split_batch_output(bwt.cpu().numpy(), term.cpu().numpy().view(np.uint64), cols)
    for c, (b, t) in zip(cols, outs):
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(b, eb) and np.array_equal(t, et)
    assert (cxbwt.get_tuning(), cxbwt.get_schedule()) == before
