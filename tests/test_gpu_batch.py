"""Batched builds: every collection of a batch equals its build alone.

Each collection's slice of cxbwt_build_batch output is compared bit for bit
with the oracle on that collection alone and with cxbwt_build on that
collection alone.
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


def _check_batch(cols, label, alone=True):
    _say(f"{label}: {len(cols)} collections, {sum(c.n_bases for c in cols)} bases")
    outs = cxbwt.build_batch_host(cols)
    for i, (c, (b, t)) in enumerate(zip(cols, outs)):
        eb, et = oracle.bwt(c.text, c.offsets)
        assert np.array_equal(b, eb), f"{label}: collection {i} BWT differs from the oracle"
        assert np.array_equal(t, et), f"{label}: collection {i} term_pos differs from the oracle"
        if alone:
            ab, at = cxbwt.build_host(c.text, c.offsets)
            assert np.array_equal(b, ab) and np.array_equal(t, at), f"{label}: collection {i} differs alone"


def test_batch_of_mixed_sizes():
    rng = np.random.default_rng(21)
    cols = []
    for k in range(24):
        kind = k % 4
        if kind == 0:
            cols.append(datagen.random_collection(rng, int(rng.integers(1, 20)), [0, 1, 5, 16, 27, 28, 29, 54, 57]))
        elif kind == 1:
            g = datagen.random_genome(rng, 5000)
            cols.append(datagen.sample_reads(rng, g, int(rng.integers(50, 400)), 100, 0.01))
        elif kind == 2:
            cols.append(datagen.from_reads(["ACGT" * 10] * int(rng.integers(1, 80))))
        else:
            cols.append(datagen.from_reads([""] * 3 + ["A"] + [""]))
    _check_batch(cols, "mixed")


def test_single_collection_batch_equals_build():
    col = datagen.plain_config(0, scale=0.2)
    _check_batch([col], "one collection")


def test_batch_shaped_like_the_batched_workload():
    cols = datagen.batch_collections(count=12, scale=0.01)
    _check_batch(cols, "batch recipe x0.01", alone=False)


def test_batch_repeat_runs_identical():
    cols = datagen.batch_collections(count=6, scale=0.005)
    _say("batch determinism")
    a = cxbwt.build_batch_host(cols)
    b = cxbwt.build_batch_host(cols)
    for (x, y), (u, v) in zip(a, b):
        assert np.array_equal(x, u) and np.array_equal(y, v)


def _largest_recipe_collections(k=None, above_bases=None):
    """Indices of the batched workload's largest collections at full size:
    the k largest, or the fewest largest whose bases pass above_bases."""
    spec = datagen.batch_specs()
    order = sorted(range(len(spec)), key=lambda j: -spec[j][0] * spec[j][1])
    if k is not None:
        return order[:k]
    out, tot = [], 0
    for j in order:
        out.append(j)
        tot += spec[j][0] * spec[j][1]
        if tot > above_bases:
            return out
    return out


def _check_with_checker(cols, outs, label):
    for i, (c, (b, t)) in enumerate(zip(cols, outs)):
        rc = oracle.check_bwt(b, t, c.text, c.offsets)
        assert rc == 0, f"{label}: collection {i} ({c.n_bases} bases) fails invariant {rc}"


def test_largest_recipe_collections_at_full_size_in_one_batch():
    """The 8 largest collections the batched recipe draws (up to 2M reads x
    150 bases, 2.06 Gbases together) in one batch at full size; each checked
    by the oracle's compiled checker, the smallest also by the full oracle."""
    idx = _largest_recipe_collections(k=8)
    cols = [datagen.batch_collection(j) for j in idx]
    _say(f"recipe-size batch: collections {idx}, {sum(c.n_bases for c in cols)} bases")
    outs = cxbwt.build_batch_host(cols)
    _check_with_checker(cols, outs, "recipe-size batch")
    small = min(range(len(cols)), key=lambda i: cols[i].n_bases)
    eb, et = oracle.bwt(cols[small].text, cols[small].offsets)
    assert np.array_equal(outs[small][0], eb) and np.array_equal(outs[small][1], et)


def test_batch_beyond_32bit_positions_in_waves():
    """Recipe collections whose bases pass 2^32 together: serve.plan_waves
    cuts them into waves below the 32-bit position limit, each wave one
    batched build; every collection checked by the compiled checker."""
    from paper_1401_7457_amd import serve
    idx = _largest_recipe_collections(above_bases=(1 << 32) + (1 << 28))
    cols = [datagen.batch_collection(j) for j in idx]
    total = sum(c.n_bases for c in cols)
    waves = serve.plan_waves([(c.n_reads, c.n_bases, c.max_read_len) for c in cols])
    _say(f"multi-wave batch: {len(cols)} collections, {total} bases, {len(waves)} waves")
    assert total > (1 << 32) and len(waves) >= 2
    for w in waves:
        part = [cols[i] for i in w]
        assert sum(c.n_bases for c in part) < (1 << 32)
        _say(f"wave of {len(part)} collections, {sum(c.n_bases for c in part)} bases")
        outs = cxbwt.build_batch_host(part)
        _check_with_checker(part, outs, "multi-wave batch")
