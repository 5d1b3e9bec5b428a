"""Builds captured in a hipGraph and replayed (cxbwt_graph_*).

Every replay is compared bit for bit with the oracle, with eager builds and
host synchronisation between replays, and with new read contents of the
same shape in the captured buffers.  The schedule inside the graph is cut
short on purpose (few captured levels; a level too large for the scratch)
so that the host's completion of the remaining levels is exercised too.
"""
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


def _device_inputs(text, offsets):
    import torch
    t_dev = torch.from_numpy(np.ascontiguousarray(text, dtype=np.uint8)).cuda()
    o_dev = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).cuda()
    packed, status = cxbwt.pack(t_dev)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return packed, o_dev


def _refill(g, text, offsets):
    """New contents for the captured input buffers (same sizes)."""
    import torch
    packed, o_dev = _device_inputs(text, offsets)
    g.packed.copy_(packed)
    g.offsets.copy_(o_dev)
    torch.cuda.synchronize()


def _expect(label, got_b, got_t, text, offsets):
    eb, et = oracle.bwt(text, offsets)
    if not np.array_equal(got_b, eb):
        bad = np.flatnonzero(got_b != eb)
        raise AssertionError(f"{label}: {bad.size} BWT rows differ, first {bad[:10].tolist()}")
    assert np.array_equal(got_t, et), f"{label}: term_pos differs"


def _replay(g, label, text, offsets):
    import torch
    _say(f"{label}: replay")
    b, t = g.run()
    torch.cuda.synchronize()
    _expect(label, b.cpu().numpy(), t.cpu().numpy().view(np.uint64), text, offsets)
    return cxbwt.last_stats()


def _same_shape(rng, genome, lens):
    """Reads of the given lengths sampled from a genome (same offsets)."""
    return datagen.sample_reads(rng, genome, lens.size, lens, 0.005)


@pytest.mark.parametrize("levels", [0, 1, 3])
def test_single_collection_replays(levels):
    """plain0-like reads; replays of three contents with eager builds between.

    levels 1 schedules only level 1 inside the graph and levels 3 stops
    mid-way; 0 schedules enough levels for any input.
    """
    import torch
    rng = np.random.default_rng(100 + levels)
    lens = rng.integers(60, 121, size=6000)
    g1, g2 = datagen.random_genome(rng, 40_000), datagen.random_genome(rng, 40_000)
    cols = [_same_shape(np.random.default_rng(7), g1, lens), _same_shape(np.random.default_rng(8), g2, lens),
            _same_shape(np.random.default_rng(9), g1, lens)]
    assert all(np.array_equal(c.offsets, cols[0].offsets) for c in cols)
    c0 = cols[0]
    packed, o_dev = _device_inputs(c0.text, c0.offsets)
    _say(f"graph levels={levels}: capture, reads={c0.n_reads} bases={c0.n_bases}")
    g = cxbwt.BuildGraph(packed, o_dev, c0.n_reads, c0.n_bases, c0.max_read_len, levels=levels)
    try:
        for k, c in enumerate(cols + cols[:1]):
            _refill(g, c.text, c.offsets)
            st = _replay(g, f"levels={levels} content {k}", c.text, c.offsets)
            _say(f"levels={levels} content {k}: stats levels={st['levels']} chunks={st['chunks']}")
            # eager work on the same device between replays
            eb, et = cxbwt.build_host(cols[1].text, cols[1].offsets)
            torch.cuda.synchronize()
            assert eb.size == cols[1].n_bases + cols[1].n_reads
    finally:
        g.close()


def test_graph_stats_match_eager_build():
    rng = np.random.default_rng(31)
    c = datagen.sample_reads(rng, datagen.random_genome(rng, 50_000), 8000, 100, 0.005)
    eb, et = cxbwt.build_host(c.text, c.offsets)
    est = cxbwt.last_stats()
    packed, o_dev = _device_inputs(c.text, c.offsets)
    g = cxbwt.BuildGraph(packed, o_dev, c.n_reads, c.n_bases, c.max_read_len)
    try:
        st = _replay(g, "stats", c.text, c.offsets)
    finally:
        g.close()
    for k in ("levels", "max_window", "chunks", "big_segments", "final_big", "chunk_suffixes", "level_suffixes",
              "scattered_suffixes", "regathered", "window_fetches"):
        assert st[k] == est[k], (k, st[k], est[k])


def test_level_too_large_for_one_batch_finishes_on_host():
    """~2000x coverage of a 1.5 kb genome: a level with more segments than the
    per-segment scratch holds stops the device schedule; the host finishes."""
    rng = np.random.default_rng(21)
    g0 = datagen.random_genome(rng, 1500)
    c = datagen.sample_reads(rng, g0, 30000, 100, 0.001)
    packed, o_dev = _device_inputs(c.text, c.offsets)
    _say("stalled schedule: capture")
    g = cxbwt.BuildGraph(packed, o_dev, c.n_reads, c.n_bases, c.max_read_len)
    try:
        st = _replay(g, "stalled schedule", c.text, c.offsets)
        assert st["level_batches"] > st["levels"] - 1, "no level ran in more than one batch"
        st = _replay(g, "stalled schedule, again", c.text, c.offsets)
    finally:
        g.close()


def test_batch_graph_equals_build_batch():
    """Collections of mixed sizes (some fit one chunk, some hold empty reads)."""
    import torch
    rng = np.random.default_rng(41)
    cols = []
    for k in range(12):
        kind = k % 3
        if kind == 0:
            cols.append(datagen.random_collection(rng, int(rng.integers(1, 20)), [0, 1, 5, 16, 27, 28, 29, 54, 57]))
        elif kind == 1:
            gg = datagen.random_genome(rng, 5000)
            cols.append(datagen.sample_reads(rng, gg, int(rng.integers(50, 400)), 100, 0.01))
        else:
            cols.append(datagen.from_reads(["ACGT" * 10] * int(rng.integers(1, 80)) + [""]))
    text, offsets, coll_reads, maxlen = cxbwt.concat_collections(cols)
    n, nb = offsets.size - 1, int(offsets[-1])
    packed, o_dev = _device_inputs(text, offsets)
    _say(f"batch graph: {len(cols)} collections, {nb} bases")
    g = cxbwt.BuildGraph(packed, o_dev, n, nb, maxlen, coll_reads=coll_reads)
    try:
        for rep in range(2):
            _say(f"batch graph replay {rep}")
            b, t = g.run()
            torch.cuda.synchronize()
            outs = cxbwt.split_batch_output(b.cpu().numpy(), t.cpu().numpy().view(np.uint64), cols)
            for i, (c, (bb, tt)) in enumerate(zip(cols, outs)):
                eb, et = oracle.bwt(c.text, c.offsets)
                assert np.array_equal(bb, eb), f"replay {rep}: collection {i} BWT differs"
                assert np.array_equal(tt, et), f"replay {rep}: collection {i} term_pos differs"
    finally:
        g.close()


def test_changed_collection_bases_are_refused():
    """Moving a base from one collection to the other keeps every size but
    not the captured level-1 plan: the replay reports CXBWT_EINVAL."""
    rng = np.random.default_rng(51)
    gg = datagen.random_genome(rng, 20_000)
    a = datagen.sample_reads(rng, gg, 3000, 80, 0.005)
    b = datagen.sample_reads(rng, gg, 3000, 60, 0.005)  # shorter: the moved base keeps every read <= 80
    text, offsets, coll_reads, maxlen = cxbwt.concat_collections([a, b])
    n, nb = offsets.size - 1, int(offsets[-1])
    packed, o_dev = _device_inputs(text, offsets)
    g = cxbwt.BuildGraph(packed, o_dev, n, nb, maxlen, coll_reads=coll_reads)
    try:
        _say("plan check: unchanged")
        g.run()
        moved = offsets.copy()
        moved[int(coll_reads[1])] -= 1  # the last read of collection 0 gives a base to collection 1
        _refill(g, text, moved)
        _say("plan check: moved boundary")
        with pytest.raises(cxbwt.CxbwtError) as e:
            g.run()
        assert e.value.status == cxbwt.EINVAL
    finally:
        g.close()


@pytest.mark.parametrize("choice", [(16, 6), (6, 3), (16, 8)])
def test_replay_with_other_instantiations(choice):
    """The wide tile and the smallest tile and chunk inside a graph (persistent
    forms of their kernels), including the host's completion (levels=2)."""
    old = cxbwt.get_tuning()
    rng = np.random.default_rng(61)
    c = datagen.sample_reads(rng, datagen.random_genome(rng, 30_000), 9000, rng.integers(40, 151, size=9000), 0.005)
    try:
        cxbwt.set_tuning(*choice)
        for levels in (0, 2):
            packed, o_dev = _device_inputs(c.text, c.offsets)
            _say(f"instantiation {choice}, levels={levels}: capture")
            g = cxbwt.BuildGraph(packed, o_dev, c.n_reads, c.n_bases, c.max_read_len, levels=levels)
            try:
                _replay(g, f"instantiation {choice}, levels={levels}", c.text, c.offsets)
            finally:
                g.close()
    finally:
        cxbwt.set_tuning(*old)


def test_replay_needing_far_more_work_than_captured():
    """Captured on 6000 copies of one read (few chunks, large final groups),
    replayed on reads of a genome of the same shape (many chunks and tiles):
    the launches sized at capture loop over the extra work."""
    rng = np.random.default_rng(71)
    one = datagen.ASCII[rng.integers(0, 4, size=100)]
    text_a = np.tile(one, 6000)
    offsets = np.arange(0, text_a.size + 1, 100, dtype=np.uint64)
    b = datagen.sample_reads(rng, datagen.random_genome(rng, 60_000), 6000, 100, 0.005)
    assert np.array_equal(b.offsets, offsets)
    packed, o_dev = _device_inputs(text_a, offsets)
    _say("capture on identical reads")
    g = cxbwt.BuildGraph(packed, o_dev, 6000, text_a.size, 100)
    try:
        for k, text in enumerate((b.text, text_a, b.text)):
            _refill(g, text, offsets)
            st = _replay(g, f"more work than captured, content {k}", text, offsets)
            _say(f"content {k}: chunks={st['chunks']} final groups={st['final_big']}")
    finally:
        g.close()


def test_replay_with_invalid_offsets_reports_edata_then_recovers():
    """A replay whose offsets are invalid (a read end past the text) reports
    CXBWT_EDATA; the next replay of valid offsets is exact again."""
    rng = np.random.default_rng(81)
    c = datagen.sample_reads(rng, datagen.random_genome(rng, 20_000), 3000, 80, 0.005)
    packed, o_dev = _device_inputs(c.text, c.offsets)
    g = cxbwt.BuildGraph(packed, o_dev, c.n_reads, c.n_bases, c.max_read_len)
    try:
        bad = c.offsets.copy()
        bad[5] = np.uint64(2 ** 40)
        _refill(g, c.text, bad)
        _say("replay with an invalid offset")
        with pytest.raises(cxbwt.CxbwtError) as e:
            g.run()
        assert e.value.status == cxbwt.EDATA
        _refill(g, c.text, c.offsets)
        _replay(g, "replay after the invalid one", c.text, c.offsets)
    finally:
        g.close()


@pytest.mark.parametrize("kind", ["all_small", "all_empty"])
def test_graph_without_levels(kind):
    """Graphs with no sort level: every collection fits one chunk, or every
    read is empty (no suffix but the terminators)."""
    import torch
    rng = np.random.default_rng(91)
    if kind == "all_small":
        cols = [datagen.random_collection(rng, int(rng.integers(1, 6)), [0, 1, 5, 16, 27, 28]) for _ in range(7)]
    else:
        cols = [datagen.from_reads([""] * 5), datagen.from_reads([""] * 3)]
    text, offsets, coll_reads, maxlen = cxbwt.concat_collections(cols)
    n, nb = offsets.size - 1, int(offsets[-1])
    packed, o_dev = _device_inputs(text, offsets)
    _say(f"graph without levels ({kind}): {len(cols)} collections, {nb} bases")
    g = cxbwt.BuildGraph(packed, o_dev, n, nb, maxlen, coll_reads=coll_reads)
    try:
        for rep in range(2):
            b, t = g.run()
            torch.cuda.synchronize()
            outs = cxbwt.split_batch_output(b.cpu().numpy(), t.cpu().numpy().view(np.uint64), cols)
            for i, (c, (bb, tt)) in enumerate(zip(cols, outs)):
                eb, et = oracle.bwt(c.text, c.offsets)
                assert np.array_equal(bb, eb), f"{kind} replay {rep}: collection {i} BWT differs"
                assert np.array_equal(tt, et), f"{kind} replay {rep}: collection {i} term_pos differs"
    finally:
        g.close()
