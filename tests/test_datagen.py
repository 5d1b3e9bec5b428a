"""Seeded synthetic inputs: determinism and the shapes of the workloads."""
import numpy as np

from paper_1401_7457_amd import datagen


def test_plain_config_deterministic_and_shaped():
    a = datagen.plain_config(0)
    b = datagen.plain_config(0)
    assert np.array_equal(a.text, b.text) and np.array_equal(a.offsets, b.offsets)
    assert a.n_reads == 10_000 and a.n_bases == 1_000_000 and a.max_read_len == 100
    assert set(np.unique(a.text).tobytes()) <= set(b"ACGT")


def test_scaled_configs_keep_shape():
    c = datagen.plain_config(1, scale=0.001)
    assert c.n_reads == 4000 and c.max_read_len == 100
    d = datagen.plain_config(2, scale=0.0005)
    assert d.n_reads == 20000


def test_substitution_rate_close_to_target():
    rng = np.random.default_rng(0)
    g = datagen.random_genome(rng, 200_000)
    m = datagen.mutate(rng, g, 0.01)
    assert abs(np.mean(m != g) - 0.01) < 0.002


def test_reverse_strand_is_reverse_complement():
    rng = np.random.default_rng(5)
    g = datagen.random_genome(rng, 1000)
    col = datagen.sample_reads(rng, g, 200, 50, 0.0, both_strands=True)
    gs = datagen.ASCII[g].tobytes().decode()
    comp = str.maketrans("ACGT", "TGCA")
    for r in col.reads():
        assert r in gs or r.translate(comp)[::-1] in gs


def test_repeat_genome_has_repeats():
    rng = np.random.default_rng(3)
    g = datagen.genome_with_repeats(rng, 400_000, repeat_frac=0.1, unit_min=1000, unit_max=2000, copies=10)
    assert g.size == 400_000
    # 32-mers from repeat families occur many times
    s = datagen.ASCII[g].tobytes()
    kmers = {}
    for p in range(0, len(s) - 32, 7):
        k = s[p:p + 32]
        kmers[k] = kmers.get(k, 0) + 1
    assert max(kmers.values()) >= 3


def test_batch_and_jobs_shapes():
    cols = datagen.batch_collections(count=4, scale=0.01)
    assert len(cols) == 4
    for c in cols:
        assert c.max_read_len in (75, 100, 150)
    jobs = datagen.job_stream(count=5, rate_per_s=10.0, scale=0.001)
    assert all(j1.arrival_s < j2.arrival_s for j1, j2 in zip(jobs, jobs[1:]))
    for j in jobs:
        L = np.diff(j.collection.offsets.astype(np.int64))
        assert L.min() >= 100 and L.max() <= 250
