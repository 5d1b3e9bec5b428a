"""The build in ranges of first-window key prefixes (Section 3.1's
partitioning, Fig. 2 steps 1-3) against the oracle, bit for bit.

Budgets far below the collection size force many ranges, refinement of
oversize prefix classes by further digits, ranges small enough for one chunk
and ranges that go through the sort levels.  The full-size 400 Mbase
collection in ranges is checked with the oracle's compiled checker.
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


def _check(col, budget, label, min_ranges=1, wide=False):
    _say(f"{label}: reads={col.n_reads} bases={col.n_bases} budget={budget} wide={wide}")
    got_b, got_t = cxbwt.build_host(col.text, col.offsets, max_range_suffixes=budget, wide=wide)
    st = cxbwt.last_stats()
    exp_b, exp_t = oracle.bwt(col.text, col.offsets)
    if not np.array_equal(got_b, exp_b):
        bad = np.flatnonzero(got_b != exp_b)
        raise AssertionError(f"{label}: {bad.size} BWT rows differ, first {bad[:10].tolist()}")
    assert np.array_equal(got_t, exp_t), f"{label}: term_pos differs"
    assert st["ranges"] >= min_ranges, f"{label}: {st['ranges']} ranges"
    return st


def test_budget_above_the_collection_is_one_range():
    col = datagen.plain_config(0, scale=0.2)
    st = _check(col, col.n_bases + 10, "one range")
    assert st["ranges"] == 1


@pytest.mark.parametrize("budget", [150_000, 40_000, 7_000, 900, 300])
def test_plain0_in_many_ranges(budget):
    """1 Mbase at 10x coverage: budgets from a few ranges down to ranges
    smaller than one chunk (thousands of ranges, classes refined to three or
    more digits)."""
    col = datagen.plain_config(0)
    _check(col, budget, f"plain0 in ranges of {budget}", min_ranges=col.n_bases // budget)


@pytest.mark.parametrize("budget", [150_000, 5_000, 300])
def test_plain0_in_ranges_with_wide_positions(budget):
    """The same with 64-bit positions in a table per range (the form of
    collections above 32-bit positions), forced on a small input."""
    col = datagen.plain_config(0)
    _check(col, budget, f"plain0 wide in ranges of {budget}", min_ranges=col.n_bases // budget, wide=True)


@pytest.mark.parametrize("wide", [False, True])
def test_repeat_heavy_sample_in_ranges(wide):
    """The repeat-heavy recipe (diverged repeat copies: long shared
    prefixes, deep refinement) at scale 0.002 in ranges of 20 000."""
    col = datagen.plain_config(2, scale=0.002)
    _check(col, 20_000, "plain2@0.002 in ranges", min_ranges=col.n_bases // 20_000, wide=wide)


def _largest_full_window_class(col) -> int:
    """Most suffixes sharing a whole first window of 27 bases (host, brute
    force).  Such a class cannot be split by first-window keys; a class of
    identical shorter suffixes can, by read order."""
    from collections import Counter
    c = Counter()
    for r in col.reads():
        for k in range(len(r) - 26):
            c[r[k:k + 27]] += 1
    return max(c.values()) if c else 0


def test_ragged_and_empty_reads_in_ranges():
    rng = np.random.default_rng(31)
    for case in range(8):
        col = datagen.random_collection(rng, int(rng.integers(1, 600)), [0, 1, 2, 5, 26, 27, 28, 53, 54, 55, 120, 300])
        if col.n_bases == 0:
            continue
        budget = int(rng.integers(1, max(2, col.n_bases // 3)))
        if _largest_full_window_class(col) > budget:
            _say(f"ragged case {case}: budget {budget} below a class of identical first windows")
            with pytest.raises(cxbwt.CxbwtError) as e:
                cxbwt.build_host(col.text, col.offsets, max_range_suffixes=budget)
            assert e.value.status == cxbwt.ERANGE
            budget = _largest_full_window_class(col)
        _check(col, budget, f"ragged case {case}", wide=bool(case % 2))


def test_identical_first_windows_beyond_the_budget_is_erange():
    rng = np.random.default_rng(60)
    read = "".join("ACGT"[x] for x in rng.integers(0, 4, size=60))  # no 27-mer twice in the read
    col = datagen.from_reads([read] * 300)
    assert _largest_full_window_class(col) == 300
    _say("identical reads, budget below one key class")
    with pytest.raises(cxbwt.CxbwtError) as e:
        cxbwt.build_host(col.text, col.offsets, max_range_suffixes=100)
    assert e.value.status == cxbwt.ERANGE
    # a budget that holds the class works, and matches the oracle
    _check(col, 300, "identical reads, budget = copies")


@pytest.mark.parametrize("wide", [False, True])
def test_homopolymers_in_ranges(wide):
    """Homopolymer reads: 700 suffixes share the whole first window AAA..A
    (budget exactly that); the shorter A and C runs are classes of identical
    suffixes cut in read order."""
    col = datagen.from_reads(["A" * 40] * 50 + ["C" * 3] * 10 + [""] * 4)
    budget = _largest_full_window_class(col)
    assert budget == 50 * 14
    _check(col, budget, "homopolymers", wide=wide)
    with pytest.raises(cxbwt.CxbwtError) as e:
        cxbwt.build_host(col.text, col.offsets, max_range_suffixes=budget - 1, wide=wide)
    assert e.value.status == cxbwt.ERANGE


@pytest.mark.parametrize("wide", [False, True])
def test_identical_short_suffixes_cut_by_read_order(wide):
    """2000 reads of 20 random bases: every class of identical suffixes (one
    per read, all shorter than a window) is far above the budget of 150 and is
    cut into ranges in read order."""
    rng = np.random.default_rng(12)
    col = datagen.from_reads(["".join("ACGT"[x] for x in rng.integers(0, 4, size=20))] * 2000 +
                             ["".join("ACGT"[x] for x in rng.integers(0, 4, size=20)) for _ in range(30)])
    _check(col, 150, "identical short suffixes", min_ranges=col.n_bases // 150, wide=wide)


def test_long_reads_in_ranges():
    """Reads of 150-1000 bases: many later windows per tied suffix, fetched
    through the position table in the wide form."""
    rng = np.random.default_rng(5)
    genome = datagen.random_genome(rng, 20_000)
    col = datagen.sample_reads(rng, genome, 400, rng.integers(150, 1001, size=400), 0.002)
    for wide in (False, True):
        _check(col, 9_000, "long reads", min_ranges=col.n_bases // 9_000, wide=wide)


def test_plain1_full_size_in_ranges():
    """4M reads x 100 bases (400 Mbases) in ranges of 50M suffixes, checked
    by the oracle's compiled checker (counts, bare-terminator rows, LF walk
    of every read)."""
    col = datagen.plain_config(1)
    _say(f"plain1 full in ranges: reads={col.n_reads} bases={col.n_bases}")
    b, t = cxbwt.build_host(col.text, col.offsets, max_range_suffixes=50_000_000)
    st = cxbwt.last_stats()
    _say(f"plain1 full in ranges: {st['ranges']} ranges, checking")
    assert st["ranges"] >= 8
    rc = oracle.check_bwt(b, t, col.text, col.offsets)
    assert rc == 0, f"plain1 in ranges: invariant {rc} fails"


def test_collection_above_32bit_positions_in_ranges():
    """45M reads x 100 bases (4.5 Gbases, above the 2^32 - 1 positions of a
    build in one piece) from a 225 Mb genome at 20x, built in three ranges
    with 64-bit positions, checked by the oracle's compiled checker."""
    col = datagen.plain_config(1, scale=11.25)
    assert col.n_bases > cxbwt.MAX_BASES
    _say(f"above 32-bit positions: reads={col.n_reads} bases={col.n_bases}")
    b, t = cxbwt.build_host(col.text, col.offsets, max_range_suffixes=1_600_000_000)
    st = cxbwt.last_stats()
    _say(f"above 32-bit positions: {st['ranges']} ranges, checking")
    assert st["ranges"] >= 3
    rc = oracle.check_bwt(b, t, col.text, col.offsets)
    assert rc == 0, f"4.5 Gbases in ranges: invariant {rc} fails"
