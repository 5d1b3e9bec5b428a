"""The plain single-build workloads at their full sizes, on the device.

Too large for the comparison-sort oracle, so the output is checked by
properties that fix the BWT completely: the symbol counts, the
bare-terminator rows, and the LF walk of every read, which must spell the
read backwards and end on its term_pos row (the compiled checker in the
oracle, pinned against true and damaged BWTs in the oracle tests).
Collected after the parity tests: these are the slowest GPU tests.
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
    cxbwt.lib()  # fail loudly if the library is missing


def _full(k):
    col = datagen.plain_config(k)
    _say(f"plain{k} full: reads={col.n_reads} bases={col.n_bases}")
    b, t = cxbwt.build_host(col.text, col.offsets)
    _say(f"plain{k} full: built, checking counts / terminator rows / LF walks")
    rc = oracle.check_bwt(b, t, col.text, col.offsets)
    assert rc == 0, f"plain{k} full size: invariant {rc} fails"
    _say(f"plain{k} full: ok")


def test_plain1_full_size():
    """4M reads x 100 bases from a 20 Mb genome (400 Mbases)."""
    _full(1)


def test_plain2_full_size_repeat_heavy():
    """40M reads x 100 bases from a 200 Mb genome with repeat families (4 Gbases)."""
    _full(2)


def test_final_groups_beyond_segment_slots():
    """3000 distinct 30-base reads, each present 520 times (46.8 Mbases).

    Every suffix shorter than a window is shared by at least 520 identical
    copies, more than the largest chunk, so it is finished as a final group:
    about 60 000 groups, more than the per-level segment slots (one per 2049
    bases), whose tile prefixes must still fit.
    """
    rng = np.random.default_rng(77)
    distinct = datagen.ASCII[rng.integers(0, 4, size=(3000, 30))]
    text = np.ascontiguousarray(np.tile(distinct, (520, 1))).reshape(-1)
    offsets = np.arange(0, text.size + 1, 30, dtype=np.uint64)
    _say(f"duplicates: reads={offsets.size - 1} bases={text.size}")
    b, t = cxbwt.build_host(text, offsets)
    st = cxbwt.last_stats()
    _say(f"duplicates: built, final groups {st['final_big']}, checking")
    assert st["final_big"] > text.size // 2049
    rc = oracle.check_bwt(b, t, text, offsets)
    assert rc == 0, f"duplicates: invariant {rc} fails"
