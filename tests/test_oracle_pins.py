"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

Every check here is independent of the oracle's own code path:
  * the worked example printed in Fig. 1 (Section 2);
  * brute force over explicit symbol tuples (exhaustive on tiny inputs);
  * the suffix array of the concatenation S_0 S_1 ... with distinct integer
    sentinels, built by prefix doubling (a textbook suffix-sorting method);
  * closed forms: one read = the classic rotation-sort BWT; n identical
    reads; homopolymers;
  * invariants: symbol counts, the bare-terminator rows, the LF-walk inverse.
Mutation tests plant plausible mistakes in a copy of the oracle source and
require that some pin fails.
"""
import itertools
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from conftest import ROOT, load_golden
from oracle import invariants, oracle
from paper_1401_7457_amd import datagen


def _col(reads):
    c = datagen.from_reads(reads)
    return c.text, c.offsets


# ---- Fig. 1 -----------------------------------------------------------------

def test_fig1_worked_example():
    g = load_golden("fig1.txt")
    text, off = _col(g["reads"])
    bwt, tp = oracle.bwt(text, off)
    assert bwt.tobytes().decode() == g["bwt"][0]
    assert tp.tolist() == [int(x) for x in g["term_pos"]]
    pairs = oracle.sorted_suffixes(text, off)
    shown = [g["reads"][i][k:] + "$" for i, k in pairs.tolist()]
    assert shown == g["suffixes"]


def test_fig1_bruteforce_agrees():
    g = load_golden("fig1.txt")
    b, tp = oracle.bwt_bruteforce(g["reads"])
    assert b == g["bwt"][0]
    assert tp == [int(x) for x in g["term_pos"]]


# ---- brute force --------------------------------------------------------------

def _all_strings(alpha, maxlen):
    for L in range(maxlen + 1):
        for t in itertools.product(alpha, repeat=L):
            yield "".join(t)


def test_exhaustive_tiny_over_AC():
    small = list(_all_strings("AC", 4))   # 31 strings
    tiny = list(_all_strings("AC", 2))    # 7 strings
    cases = [[a] for a in small] + [[a, b] for a in small for b in small]
    cases += [[a, b, c] for a in tiny for b in tiny for c in tiny]
    for reads in cases:
        text, off = _col(reads)
        bwt, tp = oracle.bwt(text, off, threads=1)
        eb, etp = oracle.bwt_bruteforce(reads)
        assert bwt.tobytes().decode() == eb, reads
        assert tp.tolist() == etp, reads


@pytest.mark.parametrize("alpha", ["A", "AC", "ACGT"])
def test_random_tiny_vs_bruteforce(alpha):
    rng = np.random.default_rng(7 + len(alpha))
    for _ in range(300):
        n = int(rng.integers(1, 7))
        reads = ["".join(rng.choice(list(alpha), size=int(rng.integers(0, 12)))) for _ in range(n)]
        text, off = _col(reads)
        for threads in (1, 3):
            bwt, tp = oracle.bwt(text, off, threads=threads)
            eb, etp = oracle.bwt_bruteforce(reads)
            assert bwt.tobytes().decode() == eb, reads
            assert tp.tolist() == etp, reads


# ---- suffix array of the concatenation, by prefix doubling ------------------

def _sa_prefix_doubling(s: np.ndarray) -> np.ndarray:
    """Suffix array of an integer string by prefix doubling (Manber & Myers)."""
    n = s.size
    rank = s.astype(np.int64)
    sa = np.arange(n)
    h = 1
    while True:
        second = np.full(n, -1, dtype=np.int64)
        second[: n - h] = rank[h:] if h < n else second[:0]
        sa = np.lexsort((second, rank))
        key = np.stack([rank[sa], second[sa]], axis=1)
        diff = np.any(key[1:] != key[:-1], axis=1)
        new = np.empty(n, dtype=np.int64)
        new[sa] = np.concatenate([[0], np.cumsum(diff)])
        rank = new
        if rank.max() == n - 1:
            return sa
        h *= 2


def _bwt_via_concatenation(reads):
    """BWT from the suffix array of S_0 $_0 S_1 $_1 ... over integers.

    $_i -> i (so terminators are distinct, ordered by read index and below
    every base), bases -> n + rank(A<C<G<T).  A comparison of two suffixes of
    the concatenation is decided at or before the first terminator, which
    makes its suffix order the multi-string order.
    """
    n = len(reads)
    rank = {"A": 0, "C": 1, "G": 2, "T": 3}
    sym, src = [], []
    for i, r in enumerate(reads):
        sym += [n + rank[c] for c in r] + [i]
        src += list(r) + ["$"]
    sa = _sa_prefix_doubling(np.array(sym, dtype=np.int64))
    starts = set()
    p = 0
    for r in reads:
        starts.add(p)
        p += len(r) + 1
    out = []
    term = [0] * n
    read_of_start = {}
    p = 0
    for i, r in enumerate(reads):
        read_of_start[p] = i
        p += len(r) + 1
    for row, pos in enumerate(sa.tolist()):
        if pos in starts:
            out.append("$")
            term[read_of_start[pos]] = row
        else:
            out.append(src[pos - 1])
    return "".join(out), term


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_oracle_matches_concatenation_suffix_array(seed):
    rng = np.random.default_rng(seed)
    col = datagen.random_collection(rng, 300, [0, 1, 2, 5, 17, 28, 29, 30, 57, 100])
    reads = col.reads()
    # add exact duplicates and shared prefixes to exercise terminator ties
    reads = reads + reads[:40] + [r[:10] for r in reads[40:80]]
    text, off = _col(reads)
    bwt, tp = oracle.bwt(text, off, threads=4)
    eb, etp = _bwt_via_concatenation(reads)
    assert bwt.tobytes().decode() == eb
    assert tp.tolist() == etp


# ---- closed forms -----------------------------------------------------------------

def _rotation_bwt(r: str):
    """Textbook BWT of a single string r$ by sorting its rotations ($ smallest)."""
    s = r + "\0"  # NUL stands for $ and sorts below A/C/G/T
    rots = sorted(range(len(s)), key=lambda k: s[k:] + s[:k])
    last = "".join(s[k - 1] for k in rots).replace("\0", "$")
    return last, rots.index(0)


@pytest.mark.parametrize("r", ["ACGT", "GATTACA", "AAAAAC", "TTTTT", "ACACACAC", "CGTACGTTAGCA" * 3, ""])
def test_single_read_is_rotation_bwt(r):
    text, off = _col([r])
    bwt, tp = oracle.bwt(text, off)
    eb, row0 = _rotation_bwt(r)
    assert bwt.tobytes().decode() == eb
    assert tp.tolist() == [row0]


@pytest.mark.parametrize("r,n", [("ACGT", 5), ("GATTACA", 3), ("CCCA", 7), ("", 4)])
def test_identical_reads_closed_form(r, n):
    single, row0 = _rotation_bwt(r)
    text, off = _col([r] * n)
    bwt, tp = oracle.bwt(text, off, threads=2)
    assert bwt.tobytes().decode() == "".join(ch * n for ch in single)
    assert tp.tolist() == [row0 * n + i for i in range(n)]


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (7, 3), (40, 9)])
def test_homopolymer_closed_form(m, n):
    text, off = _col(["A" * m] * n)
    bwt, tp = oracle.bwt(text, off)
    assert bwt.tobytes().decode() == "A" * (n * m) + "$" * n
    assert tp.tolist() == [n * m + i for i in range(n)]


# ---- invariants at moderate size ------------------------------------------------

def test_invariants_on_simulated_reads():
    col = datagen.plain_config(0, scale=0.2)
    bwt, tp = oracle.bwt(col.text, col.offsets)
    invariants.check_counts(bwt, tp, col.text, col.offsets)
    invariants.check_dollar_rows(bwt, col.text, col.offsets)
    invariants.lf_reconstruct(bwt, tp, col.text, col.offsets)


def test_thread_count_does_not_change_result():
    col = datagen.plain_config(0, scale=0.05)
    a, ta = oracle.bwt(col.text, col.offsets, threads=1)
    b, tb = oracle.bwt(col.text, col.offsets, threads=7)
    assert np.array_equal(a, b) and np.array_equal(ta, tb)


def test_rejects_non_acgt():
    with pytest.raises(ValueError):
        oracle.bwt(np.frombuffer(b"ACNT", np.uint8), np.array([0, 4], np.uint64))


# ---- packed input layout ----------------------------------------------------------

def test_pack_layout_pins():
    w = oracle.pack("ACGT")
    assert w.tolist() == [0x1B00000000000000, 0]
    w = oracle.pack("T" * 32 + "C")
    assert w.tolist() == [0xFFFFFFFFFFFFFFFF, 0x4000000000000000, 0]
    assert oracle.pack("").tolist() == [0]
    w = oracle.pack("G" * 31 + "A" + "G")
    assert w[0] == int("10" * 31 + "00", 2) and w[1] == 2 << 62


# ---- mutation tests: planted mistakes in the oracle must be caught ----------

MUTANTS = {
    "terminator_order_reversed": ("return (a->read < b->read) ? -1 : (a->read > b->read) ? 1 : 0;",
                                  "return (a->read < b->read) ? 1 : (a->read > b->read) ? -1 : 0;"),
    "dollar_above_bases": ("if (a_end) return -1;", "if (a_end) return 1;"),
    "preceding_symbol_off_by_one": ("bwt[row] = text[offsets[i] + k - 1];", "bwt[row] = text[offsets[i] + k];"),
    "C_G_swapped": ("case 'C': return 2;", "case 'C': return 3;"),
    "term_pos_dropped": ("term_pos[i] = row;", "term_pos[i] = row + 1;"),
}


def _pin_battery(lib):
    """Run the cheap pins against a (possibly mutated) oracle build."""
    failures = []
    g = load_golden("fig1.txt")
    text, off = _col(g["reads"])
    try:
        bwt, tp = oracle.bwt(text, off, lib=lib)
        if bwt.tobytes().decode() != g["bwt"][0] or tp.tolist() != [int(x) for x in g["term_pos"]]:
            failures.append("fig1")
    except Exception:
        failures.append("fig1-crash")
    rng = np.random.default_rng(11)
    reads = datagen.random_collection(rng, 50, [0, 3, 9, 20]).reads()
    text, off = _col(reads)
    bwt, tp = oracle.bwt(text, off, lib=lib)
    eb, etp = _bwt_via_concatenation(reads)
    if bwt.tobytes().decode() != eb or tp.tolist() != etp:
        failures.append("concat-sa")
    return failures


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "cx_oracle.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "mut.c")
        with open(p, "w") as f:
            f.write(src.replace(old, new))
        so = oracle.compile_oracle(p, os.path.join(d, "libmut.so"))
        lib = oracle.load(so)
        assert _pin_battery(lib), f"planted mistake '{name}' passed every pin"


def test_unmutated_oracle_passes_battery():
    assert _pin_battery(oracle.load()) == []


# ---- the compiled invariant checker (used on full-size device outputs) ----

def test_c_checker_accepts_true_bwts_and_rejects_damaged_ones():
    col = datagen.plain_config(0, scale=0.3)
    bwt, tp = oracle.bwt(col.text, col.offsets)
    assert oracle.check_bwt(bwt, tp, col.text, col.offsets, threads=3) == 0
    rng = np.random.default_rng(2)
    # swap two different symbols: counts hold, the LF walk does not
    for _ in range(5):
        b = bwt.copy()
        i, j = rng.integers(col.n_reads, b.size, size=2)
        while b[i] == b[j]:
            j = rng.integers(col.n_reads, b.size)
        b[i], b[j] = b[j], b[i]
        assert oracle.check_bwt(b, tp, col.text, col.offsets) != 0
    b = bwt.copy()
    b[5] = ord("A") if b[5] != ord("A") else ord("C")
    assert oracle.check_bwt(b, tp, col.text, col.offsets) != 0
    t = tp.copy()
    t[0], t[1] = t[1], t[0]
    assert oracle.check_bwt(bwt, t, col.text, col.offsets) != 0


def test_c_checker_on_edge_collections():
    for reads in (["ACGT", "TAGT", "GGAA"], ["", "A", ""], ["A" * 30] * 4, ["ACGTACGT"]):
        c = datagen.from_reads(reads)
        b, t = oracle.bwt(c.text, c.offsets)
        assert oracle.check_bwt(b, t, c.text, c.offsets) == 0


# ---- live-round profile (ties left after each window) -----------------------

def _tied_bruteforce(reads, width):
    """Per round r, suffixes that share their first r*width bases with another."""
    sufs = [r[k:] for r in reads for k in range(len(r) + 1)]
    out = []
    r = 1
    while True:
        need = r * width
        heads = [s[:need] for s in sufs if len(s) >= need]
        seen = {}
        for h in heads:
            seen[h] = seen.get(h, 0) + 1
        c = sum(v for v in seen.values() if v > 1)
        if c == 0:
            return out
        out.append(c)
        r += 1


@pytest.mark.parametrize("alpha", ["A", "AC", "ACGT"])
def test_live_profile_vs_pairwise_bruteforce(alpha):
    rng = np.random.default_rng(31 + len(alpha))
    for _ in range(200):
        n = int(rng.integers(1, 8))
        reads = ["".join(rng.choice(list(alpha), size=int(rng.integers(0, 14)))) for _ in range(n)]
        text, off = _col(reads)
        for width in (1, 2, 3, 5):
            assert oracle.live_profile(text, off, width) == _tied_bruteforce(reads, width), (reads, width)


def test_live_profile_closed_forms():
    # n identical reads of length m: after r windows every suffix with at
    # least r*w bases is tied with its copies, (n)(m - r*w + 1) of them
    text, off = _col(["ACGTTGCA"] * 4)
    assert oracle.live_profile(text, off, 3) == [4 * 6, 4 * 3]
    # one homopolymer read A^m: after r windows the m - r*w + 1 suffixes with
    # at least r*w bases all share them, while two or more are left
    text, off = _col(["A" * 8])
    assert oracle.live_profile(text, off, 2) == [7, 5, 3]
    assert oracle.live_profile(text, off, 4) == [5]
    # distinct reads with no shared 2-base prefix
    text, off = _col(["AC", "GT", "CA"])
    assert oracle.live_profile(text, off, 2) == []
    # the adjacent common prefixes of Fig. 1's collection by hand
    reads = ["ACG", "AC"]
    text, off = _col(reads)
    order = oracle.sorted_suffixes(text, off)
    assert oracle.adjacent_lcp(text, off, order).tolist() == _lcp_by_hand(reads, order)


def _lcp_by_hand(reads, order):
    sufs = [reads[i][k:] for i, k in order.tolist()]
    out = [0]
    for x, y in zip(sufs, sufs[1:]):
        c = 0
        while c < min(len(x), len(y)) and x[c] == y[c]:
            c += 1
        out.append(c)
    return out


# ---- the Python invariant checks reject damaged BWTs ------------------------
# Each damage below keeps everything the other checks look at, so the check
# named in the test is the one that must catch it; a check that accepted
# everything would fail here.

def _small_true_bwt():
    col = datagen.plain_config(0, scale=0.05)
    bwt, tp = oracle.bwt(col.text, col.offsets)
    return col, bwt, tp


def _swap_rows_with_different_symbols(bwt, lo, rng):
    b = bwt.copy()
    i = int(rng.integers(lo, b.size))
    j = int(rng.integers(lo, b.size))
    while b[i] == b[j]:
        j = int(rng.integers(lo, b.size))
    b[i], b[j] = b[j], b[i]
    return b


def test_check_counts_rejects_wrong_symbols_and_term_pos():
    col, bwt, tp = _small_true_bwt()
    invariants.check_counts(bwt, tp, col.text, col.offsets)
    b = bwt.copy()
    i = col.n_reads + 7
    b[i] = ord("A") if b[i] != ord("A") else ord("C")
    with pytest.raises(AssertionError):
        invariants.check_counts(b, tp, col.text, col.offsets)
    b = bwt.copy()
    b[int(tp[3])] = ord("G")  # a '$' row loses its terminator
    with pytest.raises(AssertionError):
        invariants.check_counts(b, tp, col.text, col.offsets)
    t = tp.copy()
    t[0] = next(r for r in range(col.n_reads, bwt.size) if bwt[r] != ord("$"))
    with pytest.raises(AssertionError):
        invariants.check_counts(bwt, t, col.text, col.offsets)


def test_check_dollar_rows_rejects_moved_terminator_rows():
    col, bwt, tp = _small_true_bwt()
    invariants.check_dollar_rows(bwt, col.text, col.offsets)
    # rows 0 and 1 exchanged (their symbols differ): counts still hold
    k = next(k for k in range(col.n_reads - 1) if bwt[k] != bwt[k + 1])
    b = bwt.copy()
    b[k], b[k + 1] = b[k + 1], b[k]
    invariants.check_counts(b, tp, col.text, col.offsets)
    with pytest.raises(AssertionError):
        invariants.check_dollar_rows(b, col.text, col.offsets)
    # a bare-terminator row exchanged with a later row of another symbol
    j = next(j for j in range(col.n_reads, bwt.size) if bwt[j] != bwt[0] and bwt[j] != ord("$"))
    b = bwt.copy()
    b[0], b[j] = b[j], b[0]
    with pytest.raises(AssertionError):
        invariants.check_dollar_rows(b, col.text, col.offsets)


def test_lf_reconstruct_rejects_swapped_symbols_and_term_pos():
    col, bwt, tp = _small_true_bwt()
    invariants.lf_reconstruct(bwt, tp, col.text, col.offsets)
    rng = np.random.default_rng(5)
    for _ in range(5):
        b = _swap_rows_with_different_symbols(bwt, col.n_reads, rng)
        invariants.check_counts(b, tp, col.text, col.offsets)
        invariants.check_dollar_rows(b, col.text, col.offsets)
        with pytest.raises(AssertionError):
            invariants.lf_reconstruct(b, tp, col.text, col.offsets)
    # term_pos entries of two reads exchanged: still the set of '$' rows
    t = tp.copy()
    t[0], t[1] = t[1], t[0]
    invariants.check_counts(bwt, t, col.text, col.offsets)
    with pytest.raises(AssertionError):
        invariants.lf_reconstruct(bwt, t, col.text, col.offsets)
    # the walk of one listed read only
    with pytest.raises(AssertionError):
        invariants.lf_reconstruct(bwt, t, col.text, col.offsets, reads=np.array([1]))
    invariants.lf_reconstruct(bwt, t, col.text, col.offsets, reads=np.array([2, 3]))


# ---- the C oracle under AddressSanitizer + UndefinedBehaviorSanitizer -------

def test_oracle_c_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-pthread", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), os.path.join(ROOT, "oracle", "cx_oracle.c"),
           "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "asan" in (res.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + res.stderr[-200:])
    assert res.returncode == 0, res.stderr
    # verify_asan_link_order=0: the process may start with other libraries preloaded
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "runtime error" not in run.stderr
    assert "oracle sanitizer run ok" in run.stdout
