"""Window loads made by the device build against the oracle's tie profile.

Sorting by successive 27-base windows and refining only tied suffixes
(Section 3.2's stringword iterations, restricted to the suffixes still
undecided) loads window r of a suffix exactly when some other suffix shares
its first 27 r bases.  The oracle counts those suffixes from the common
prefixes of neighbouring rows of its own sort; the device reports the loads
it made, inside waves and by the global levels.  The two totals must agree
exactly: a schedule that loaded more would be doing redundant work, one that
loaded fewer could not have ordered the ties.
"""
import sys

import numpy as np
import pytest

from oracle import oracle
from paper_1401_7457_amd import cxbwt, datagen

pytestmark = pytest.mark.gpu

WINDOW_BASES = 27  # bases per key window of the device build


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    cxbwt.lib()  # fail loudly if the library is missing


def _copies():
    # 3000 copies of one 100-base read among random reads: one tied family far
    # larger than a wave's chunk, refined by the global levels
    rng = np.random.default_rng(1401)
    base = datagen.random_collection(rng, 4000, [60, 100, 150])
    one = base.text[:100].tobytes().decode() if base.n_bases >= 100 else "ACGT" * 25
    reads = base.reads() + [one] * 3000
    order = rng.permutation(len(reads))
    return datagen.from_reads([reads[i] for i in order])


CASES = {
    "plain0": lambda: datagen.plain_config(0),
    "plain2@0.002": lambda: datagen.plain_config(2, scale=0.002),
    "copies": _copies,
}


@pytest.mark.parametrize("case", list(CASES))
def test_window_loads_equal_oracle_tie_profile(case):
    col = CASES[case]()
    _say(f"{case}: reads={col.n_reads} bases={col.n_bases}")
    b, t = cxbwt.build_host(col.text, col.offsets)
    st = cxbwt.last_stats()
    _say(f"{case}: built; fetches={st['window_fetches']} regathered={st['regathered']} "
         f"max_window={st['max_window']}")
    order = oracle.sorted_suffixes(col.text, col.offsets)
    prof = oracle.live_profile(col.text, col.offsets, WINDOW_BASES, order=order)
    _say(f"{case}: oracle tie profile {prof}")
    exp_b, exp_t = oracle.bwt(col.text, col.offsets)
    assert np.array_equal(b, exp_b) and np.array_equal(t, exp_t)
    assert st["window_fetches"] + st["regathered"] == sum(prof)


def test_batch_window_loads_equal_sum_of_collection_profiles():
    # a suffix ties only with suffixes of its own collection: the batch's
    # loads are the sum of each collection's profile, not the profile of the
    # collections pooled
    rng = np.random.default_rng(7457)
    cols = []
    for k in range(12):
        g = datagen.random_genome(rng, int(rng.integers(2000, 20000)))
        cols.append(datagen.sample_reads(rng, g, int(rng.integers(200, 3000)), [75, 100, 150][k % 3], 0.01))
    shared = "ACGTTGCAAC" * 10
    cols.append(datagen.from_reads([shared] * 700))
    cols.append(datagen.from_reads([shared] * 5 + ["ACGT" * 20] * 3))
    _say(f"batch: {len(cols)} collections, {sum(c.n_bases for c in cols)} bases")
    outs = cxbwt.build_batch_host(cols)
    st = cxbwt.last_stats()
    total = 0
    for i, (c, (b, t)) in enumerate(zip(cols, outs)):
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(b, eb) and np.array_equal(t, et), f"collection {i} differs from the oracle"
        total += sum(oracle.live_profile(c.text, c.offsets, WINDOW_BASES))
    _say(f"batch: fetches={st['window_fetches']} regathered={st['regathered']} oracle total={total}")
    assert st["window_fetches"] + st["regathered"] == total
