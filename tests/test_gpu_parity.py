"""Device BWT against the CPU oracle, element by element (bit-exact).

Every case prints its name and shape before touching the GPU.  All device
work goes through the C ABI (paper_1401_7457_amd.cxbwt, a ctypes binding).
"""
import sys

import numpy as np
import pytest

from conftest import load_golden
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
    return torch.device("cuda")


def _check(col, label, threads=None):
    _say(f"{label}: reads={col.n_reads} bases={col.n_bases} maxlen={col.max_read_len}")
    got_b, got_t = cxbwt.build_host(col.text, col.offsets)
    exp_b, exp_t = oracle.bwt(col.text, col.offsets, threads=threads)
    if not np.array_equal(got_b, exp_b):
        bad = np.flatnonzero(got_b != exp_b)
        raise AssertionError(f"{label}: {bad.size} BWT rows differ, first {bad[:10].tolist()}")
    assert np.array_equal(got_t, exp_t), f"{label}: term_pos differs"
    return got_b, got_t


def test_fig1_on_device():
    g = load_golden("fig1.txt")
    col = datagen.from_reads(g["reads"])
    _say("fig1")
    b, t = cxbwt.build_host(col.text, col.offsets)
    assert b.tobytes().decode() == g["bwt"][0]
    assert t.tolist() == [int(x) for x in g["term_pos"]]


def test_pack_matches_layout():
    import torch
    rng = np.random.default_rng(3)
    for nb in (0, 1, 31, 32, 33, 64, 1000, 4097):
        _say(f"pack nb={nb}")
        text = datagen.ASCII[rng.integers(0, 4, size=nb)] if nb else np.zeros(0, np.uint8)
        dev = torch.from_numpy(text).cuda() if nb else torch.empty(0, dtype=torch.uint8, device="cuda")
        packed, status = cxbwt.pack(dev)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert np.array_equal(packed.cpu().numpy().view(np.uint64), oracle.pack(text))


def test_pack_flags_bad_bytes():
    import torch
    _say("pack bad byte")
    dev = torch.from_numpy(np.frombuffer(b"ACGTNACGT", np.uint8).copy()).cuda()
    _, status = cxbwt.pack(dev)
    torch.cuda.synchronize()
    assert int(status.item()) != 0
    # whole 32-byte words take the vector-load path: one bad byte anywhere in them
    rng = np.random.default_rng(5)
    for bad in (b"N", b"a", b"\x00", b"U", b"\xc1"):
        for at in (0, 31, 32, 500, 4095):
            text = datagen.ASCII[rng.integers(0, 4, size=4096)].copy()
            text[at] = bad[0]
            _say(f"pack bad byte {bad!r} at {at}")
            _, status = cxbwt.pack(torch.from_numpy(text).cuda())
            torch.cuda.synchronize()
            assert int(status.item()) != 0, (bad, at)


def test_pack_unaligned_source():
    import torch
    rng = np.random.default_rng(6)
    text = datagen.ASCII[rng.integers(0, 4, size=5000)]
    dev = torch.from_numpy(text).cuda()
    for off in (1, 3, 8, 16, 17):
        _say(f"pack unaligned offset {off}")
        packed, status = cxbwt.pack(dev[off:])
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert np.array_equal(packed.cpu().numpy().view(np.uint64), oracle.pack(text[off:]))


EDGE_LENS = [0, 1, 2, 15, 16, 17, 26, 27, 28, 29, 30, 53, 54, 55, 56, 57, 80, 81, 82, 84, 85, 100, 108, 112, 113]


@pytest.mark.parametrize("alphabet", [b"A", b"AC", b"ACGT"])
def test_tiny_fuzz(alphabet):
    rng = np.random.default_rng(len(alphabet))
    for trial in range(150):
        n = int(rng.integers(1, 40))
        col = datagen.random_collection(rng, n, EDGE_LENS, alphabet=alphabet)
        reads = col.reads()
        if trial % 3 == 0:
            reads = reads + reads[: max(1, len(reads) // 2)]  # exact duplicates
        if trial % 4 == 1:
            reads = reads + [r[: len(r) // 2] for r in reads]  # shared prefixes
        _check(datagen.from_reads(reads), f"fuzz {alphabet.decode()} #{trial}")


def test_plain0_full():
    _check(datagen.plain_config(0), "plain0 (1 Mbase)")


def test_plain1_scaled():
    _check(datagen.plain_config(1, scale=0.02), "plain1 x0.02")


def test_plain2_scaled_repeats():
    _check(datagen.plain_config(2, scale=0.002), "plain2 x0.002 (repeat families)")


def test_identical_reads_beyond_one_workgroup():
    rng = np.random.default_rng(9)
    r = datagen.ASCII[rng.integers(0, 4, size=100)].tobytes().decode()
    n = 9000  # each tie group holds 9000 suffixes: more than one workgroup
    col = datagen.from_reads([r] * n)
    b, t = _check(col, "identical reads x9000")
    single_b, single_t = oracle.bwt_bruteforce([r])
    assert b.tobytes().decode() == "".join(ch * n for ch in single_b)


@pytest.mark.parametrize("copies", [110, 140, 250, 380, 500])
def test_tie_groups_sorted_by_the_network(copies):
    """Tie groups of 110-500 suffixes inside chunks of 384 and 512 (6 and 8
    suffixes a lane), where groups above 96 are sorted by a bitonic network
    on (ordering bits, handle): families of near-identical reads (a few
    substitutions apart, so that groups split at different windows) mixed
    with their exact copies and with random reads, for both chunk sizes."""
    rng = np.random.default_rng(copies)
    base = datagen.ASCII[rng.integers(0, 4, size=120)].tobytes().decode()
    reads = []
    for k in range(copies):
        r = list(base)
        if k % 3:  # two of three copies carry one substitution past the first window
            pos = int(rng.integers(30, 120))
            r[pos] = "ACGT"[int(rng.integers(0, 4))]
        reads.append("".join(r)[: int(rng.integers(60, 121))])
    reads += [datagen.ASCII[rng.integers(0, 4, size=int(rng.integers(0, 150)))].tobytes().decode()
              for _ in range(400)]
    order = rng.permutation(len(reads))
    col = datagen.from_reads([reads[i] for i in order])
    before = (cxbwt.get_tuning(), cxbwt.get_schedule())
    try:
        for tile, chunk in ((16, 6), (8, 8)):
            cxbwt.set_tuning(tile, chunk)
            _check(col, f"tie groups of {copies}, {tile}x{chunk}")
    finally:
        cxbwt.set_tuning(*before[0])
        cxbwt.set_schedule(before[1])


def test_homopolymers_beyond_one_workgroup():
    col = datagen.from_reads(["A" * 100] * 6000 + ["C" * 57] * 5000)
    _check(col, "homopolymers")


def test_long_reads():
    rng = np.random.default_rng(12)
    g = datagen.random_genome(rng, 20000)
    col = datagen.sample_reads(rng, g, 3000, rng.integers(150, 1000, size=3000), 0.002)
    _check(col, "long reads 150-1000")


def test_high_coverage_small_genome():
    rng = np.random.default_rng(13)
    g = datagen.random_genome(rng, 3000)
    col = datagen.sample_reads(rng, g, 20000, 100, 0.001)  # ~650x coverage: large tie groups
    _check(col, "650x coverage")


def test_levels_in_several_batches():
    """~2000x coverage of a 1.5 kb genome: thousands of level-2 segments of
    more than one chunk each, more than the level scratch takes at once."""
    rng = np.random.default_rng(21)
    g = datagen.random_genome(rng, 1500)
    col = datagen.sample_reads(rng, g, 30000, 100, 0.001)
    _check(col, "2000x coverage, batched levels")
    st = cxbwt.last_stats()
    _say(f"levels={st['levels']} level_batches={st['level_batches']}")
    assert st["level_batches"] > st["levels"] - 1, "no level ran in more than one batch"


def test_variable_lengths_served_shape():
    rng = np.random.default_rng(14)
    g = datagen.random_genome(rng, 200_000)
    col = datagen.sample_reads(rng, g, 20000, rng.integers(100, 251, size=20000), 0.01)
    _check(col, "lengths 100-250")


def test_device_rejects_bad_offsets():
    import torch
    _say("bad offsets")
    text = np.frombuffer(b"ACGTACGT", np.uint8).copy()
    # huge first offsets too: a valid read must not take its output row from them
    for offs in ([0, 5, 3, 8], [1, 4, 8], [0, 4, 7], [10**12, 4, 8], [0, 2**40, 8], [2**40, 2**40 + 4, 8]):
        t = torch.from_numpy(text).cuda()
        o = torch.tensor(offs, dtype=torch.int64, device="cuda")
        packed, _ = cxbwt.pack(t)
        with pytest.raises(cxbwt.CxbwtError) as ei:
            cxbwt.build(packed, o, len(offs) - 1, 8, 8)
        assert ei.value.status == cxbwt.EDATA


def test_device_rejects_read_longer_than_declared():
    import torch
    _say("read too long")
    t = torch.from_numpy(np.frombuffer(b"ACGTACGT", np.uint8).copy()).cuda()
    o = torch.tensor([0, 2, 8], dtype=torch.int64, device="cuda")
    packed, _ = cxbwt.pack(t)
    with pytest.raises(cxbwt.CxbwtError) as ei:
        cxbwt.build(packed, o, 2, 8, 5)
    assert ei.value.status == cxbwt.EDATA


def test_repeat_runs_are_identical():
    col = datagen.plain_config(0, scale=0.3)
    _say("determinism")
    a = cxbwt.build_host(col.text, col.offsets)
    b = cxbwt.build_host(col.text, col.offsets)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
