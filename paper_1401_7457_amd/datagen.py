"""Seeded synthetic read collections shaped like the paper's workloads.

The paper measures on subsets of the YH short reads (100 bp, A/C/G/T only);
those reads are not available here, so every input is simulated: a uniform
random genome (optionally carrying diverged repeat families), reads sampled at
uniform start positions from either strand, and uniform random substitution
errors.  Reads are emitted as ASCII (A/C/G/T) concatenated, plus n+1 base
offsets, in generation order.

This module holds no part of the BWT method itself; the oracle and the device
path both take its output as plain input.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)
BASE_SEED = 14017457

_CHUNK = 1 << 18  # reads generated per vectorised chunk


def _workers() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


@dataclass
class Collection:
    text: np.ndarray     # uint8 ASCII, all reads concatenated
    offsets: np.ndarray  # uint64, n + 1 entries
    seed: int = 0
    label: str = ""

    @property
    def n_reads(self) -> int:
        return int(self.offsets.size - 1)

    @property
    def n_bases(self) -> int:
        return int(self.offsets[-1])

    @property
    def max_read_len(self) -> int:
        if self.n_reads == 0:
            return 0
        return int(np.max(np.diff(self.offsets.astype(np.int64))))

    def reads(self) -> list[str]:
        t = self.text.tobytes().decode()
        o = self.offsets
        return [t[int(o[i]):int(o[i + 1])] for i in range(self.n_reads)]


def from_reads(reads: list[str]) -> Collection:
    """Collection from an explicit list of read strings."""
    lens = np.array([len(r) for r in reads], dtype=np.uint64)
    offsets = np.zeros(len(reads) + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    text = np.frombuffer("".join(reads).encode(), dtype=np.uint8).copy()
    return Collection(text, offsets)


def random_genome(rng: np.random.Generator, length: int) -> np.ndarray:
    """Uniform i.i.d. genome as 2-bit symbol codes (uint8 0..3)."""
    return rng.integers(0, 4, size=length, dtype=np.uint8)


def mutate(rng: np.random.Generator, codes: np.ndarray, rate: float) -> np.ndarray:
    """Substitute each symbol with probability `rate` by one of the other three."""
    out = codes.copy()
    if rate <= 0 or out.size == 0:
        return out
    hit = rng.random(out.size, dtype=np.float32) < np.float32(rate)
    k = int(np.count_nonzero(hit))
    if k:
        out[hit] = (out[hit] + rng.integers(1, 4, size=k, dtype=np.uint8)) & 3
    return out


def genome_with_repeats(rng: np.random.Generator, length: int, repeat_frac: float = 0.10,
                        unit_min: int = 1000, unit_max: int = 5000, copies: int = 50,
                        divergence: float = 0.01) -> np.ndarray:
    """Random genome in which `repeat_frac` of the bases are repeat families.

    Each family is a random unit of length U ~ uniform{unit_min..unit_max}
    written `copies` times, every copy independently mutated at `divergence`;
    families are added until the requested repeat mass is covered.  The
    copies are shuffled and laid out between random-length unique gaps, which
    places them at uniform non-overlapping positions.
    """
    target = int(length * repeat_frac)
    pieces = []
    covered = 0
    while covered < target:
        u = int(rng.integers(unit_min, unit_max + 1))
        unit = random_genome(rng, u)
        for _ in range(copies):
            pieces.append(mutate(rng, unit, divergence))
        covered += u * copies
    rep_total = sum(p.size for p in pieces)
    if rep_total > length:
        raise ValueError("repeat mass exceeds genome length")
    order = rng.permutation(len(pieces))
    unique_total = length - rep_total
    cuts = np.sort(rng.integers(0, unique_total + 1, size=len(pieces)))
    gaps = np.diff(np.concatenate([[0], cuts, [unique_total]]))
    out = np.empty(length, dtype=np.uint8)
    pos = 0
    for gi, pi in zip(range(len(pieces)), order):
        g = int(gaps[gi])
        out[pos:pos + g] = random_genome(rng, g)
        pos += g
        p = pieces[pi]
        out[pos:pos + p.size] = p
        pos += p.size
    g = int(gaps[-1])
    out[pos:pos + g] = random_genome(rng, g)
    return out


def sample_reads(rng: np.random.Generator, genome: np.ndarray, n: int, read_len,
                 error_rate: float, both_strands: bool = True) -> Collection:
    """Sample n reads from `genome` (2-bit codes).

    read_len: an int (fixed length) or an array of n per-read lengths.  Start
    positions are uniform in [0, G - L]; with both_strands the read is the
    reverse complement with probability 1/2; each base is then substituted
    with probability error_rate.
    """
    G = genome.size
    lens = np.full(n, read_len, dtype=np.int64) if np.isscalar(read_len) else np.asarray(read_len, dtype=np.int64)
    if lens.size != n:
        raise ValueError("need one length per read")
    if n and lens.max() > G:
        raise ValueError("read longer than genome")
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens.astype(np.uint64), out=offsets[1:])
    text = np.empty(int(offsets[-1]), dtype=np.uint8)
    starts = rng.integers(0, G - lens + 1)
    strand = rng.random(n) < 0.5 if both_strands else np.zeros(n, dtype=bool)
    idx_t = np.int32 if G < (1 << 31) - 1 else np.int64
    # every chunk of reads draws its substitutions from a generator of its
    # own, so chunks can be filled in parallel and the result does not
    # depend on the thread count
    n_chunks = (n + _CHUNK - 1) // _CHUNK
    chunk_seeds = rng.integers(0, 1 << 63, size=n_chunks, dtype=np.int64)

    def fill(ci: int) -> None:
        c0 = ci * _CHUNK
        c1 = min(n, c0 + _CHUNK)
        L = lens[c0:c1].astype(idx_t)
        if int(L.sum()) == 0:
            return
        s = starts[c0:c1].astype(idx_t)
        rev = strand[c0:c1]
        maxL = int(L.max())
        j = np.arange(maxL, dtype=idx_t)[None, :]
        # base j of a forward read is genome[s + j]; of a reverse read, the
        # complement of genome[s + L - 1 - j]
        pos = np.where(rev[:, None], (s + L - 1)[:, None] - j, s[:, None] + j)
        valid = j < L[:, None]
        np.clip(pos, 0, G - 1, out=pos)
        codes = genome[pos]
        codes = np.where(rev[:, None], 3 - codes, codes).astype(np.uint8)
        codes = codes[valid] if maxL and not bool(valid.all()) else codes.reshape(-1)
        codes = mutate(np.random.Generator(np.random.PCG64(int(chunk_seeds[ci]))), codes, error_rate)
        b0 = int(offsets[c0])
        text[b0:b0 + codes.size] = ASCII[codes]

    workers = min(n_chunks, _workers())
    if workers <= 1:
        for ci in range(n_chunks):
            fill(ci)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(fill, range(n_chunks)))
    return Collection(text, offsets)


# --- the five workloads (plain, plain, repeat-heavy, batched, served) -------

def plain_config(k: int, scale: float = 1.0) -> Collection:
    """Plain single-collection workloads 0, 1 and 2.

    scale < 1 shrinks the read count and genome together (same coverage and
    shape) for tests that must finish quickly.
    """
    ss = np.random.SeedSequence(BASE_SEED + k)
    g_ss, r_ss = ss.spawn(2)
    if k == 0:
        G, n, L, e = 100_000, 10_000, 100, 0.01
    elif k == 1:
        G, n, L, e = 20_000_000, 4_000_000, 100, 0.005
    elif k == 2:
        G, n, L, e = 200_000_000, 40_000_000, 100, 0.005
    else:
        raise ValueError("plain workloads are 0, 1, 2")
    G = max(1000, int(G * scale))
    n = max(1, int(n * scale))
    g_rng = np.random.Generator(np.random.PCG64(g_ss))
    genome = genome_with_repeats(g_rng, G) if k == 2 else random_genome(g_rng, G)
    col = sample_reads(np.random.Generator(np.random.PCG64(r_ss)), genome, n, L, e)
    col.seed = BASE_SEED + k
    col.label = f"plain{k}" + ("" if scale == 1.0 else f"@{scale:g}")
    return col


def length_sweep_config(read_len: int, total_bases: int = 2_000_000_000, coverage: int = 20) -> Collection:
    """Reads of one length at a fixed total of bases (the read-length sweep of
    Section 4.3, Table 4: 100, 200 and 400 bp at equal bases).

    n = total_bases / read_len reads from a uniform random genome of
    total_bases / coverage bases, both strands, 0.5% substitutions.
    """
    ss = np.random.SeedSequence([BASE_SEED + 5, int(read_len)])
    g_ss, r_ss = ss.spawn(2)
    G = max(2 * read_len, total_bases // coverage)
    n = max(1, total_bases // read_len)
    genome = random_genome(np.random.Generator(np.random.PCG64(g_ss)), G)
    col = sample_reads(np.random.Generator(np.random.PCG64(r_ss)), genome, n, read_len, 0.005)
    col.seed = BASE_SEED + 5
    col.label = f"sweep{read_len}"
    return col


def batch_specs(count: int = 256, scale: float = 1.0, seed: int = BASE_SEED + 3) -> list[tuple[int, int, int]]:
    """(reads, read length, genome bases) of every collection of the batched
    workload: reads log-uniform on [5k, 2M] (times scale), read length fixed
    per collection from {75, 100, 150}, genome uniform in [1, 10] Mb (times
    scale).  Cheap: no collection is generated."""
    meta_ss = np.random.SeedSequence(seed).spawn(count + 1)[0]
    meta = np.random.Generator(np.random.PCG64(meta_ss))
    out = []
    for _ in range(count):
        n = int(round(math.exp(meta.uniform(math.log(5_000), math.log(2_000_000))) * scale))
        L = int(meta.choice([75, 100, 150]))
        G = int(meta.integers(1_000_000, 10_000_001) * scale)
        out.append((max(n, 1), L, max(G, 2 * L)))
    return out


def batch_collection(j: int, count: int = 256, scale: float = 1.0, seed: int = BASE_SEED + 3) -> Collection:
    """Collection j of the batched workload (the same as batch_collections()[j])."""
    n, L, G = batch_specs(count, scale, seed)[j]
    col_ss = np.random.SeedSequence(seed).spawn(count + 1)[1 + j]
    rng = np.random.Generator(np.random.PCG64(col_ss))
    genome = random_genome(rng, G)
    col = sample_reads(rng, genome, n, L, 0.005)
    col.seed = seed
    col.label = f"batch{j}"
    return col


def batch_collections(count: int = 256, scale: float = 1.0, seed: int = BASE_SEED + 3) -> list[Collection]:
    """Independent collections of uneven size and read length (batch_specs),
    each from its own random genome at 0.5% substitutions."""
    return [batch_collection(j, count, scale, seed) for j in range(count)]


@dataclass
class Job:
    arrival_s: float
    collection: Collection


def job_stream(count: int = 300, rate_per_s: float = 1.0, scale: float = 1.0,
               seed: int = BASE_SEED + 4) -> list[Job]:
    """Poisson job stream: exponential inter-arrival gaps at `rate_per_s`.

    Each job: log-uniform [10k, 5M] reads (times scale), per-read length
    uniform in [100, 250], its own random genome uniform in [1, 10] Mb (times
    scale), 1% substitutions.
    """
    ss = np.random.SeedSequence(seed)
    meta_ss, *job_ss = ss.spawn(count + 1)
    meta = np.random.Generator(np.random.PCG64(meta_ss))
    t = 0.0
    jobs = []
    for j in range(count):
        t += float(meta.exponential(1.0 / rate_per_s))
        n = max(1, int(round(math.exp(meta.uniform(math.log(10_000), math.log(5_000_000))) * scale)))
        G = max(500, int(meta.integers(1_000_000, 10_000_001) * scale))
        rng = np.random.Generator(np.random.PCG64(job_ss[j]))
        lens = rng.integers(100, 251, size=n)
        genome = random_genome(rng, max(G, 251))
        col = sample_reads(rng, genome, n, lens, 0.01)
        col.seed = seed
        col.label = f"job{j}"
        jobs.append(Job(t, col))
    return jobs


def random_collection(rng: np.random.Generator, n_reads: int, lengths, alphabet: bytes = b"ACGT") -> Collection:
    """Tiny fuzz collections: i.i.d. symbols from `alphabet`, given lengths.

    lengths: an int, or a sequence to draw each read's length from.
    """
    if np.isscalar(lengths):
        lens = np.full(n_reads, int(lengths), dtype=np.int64)
    else:
        lens = rng.choice(np.asarray(lengths, dtype=np.int64), size=n_reads)
    alpha = np.frombuffer(alphabet, dtype=np.uint8)
    total = int(lens.sum())
    text = alpha[rng.integers(0, alpha.size, size=total)] if total else np.zeros(0, np.uint8)
    offsets = np.zeros(n_reads + 1, dtype=np.uint64)
    np.cumsum(lens.astype(np.uint64), out=offsets[1:])
    return Collection(np.ascontiguousarray(text, dtype=np.uint8), offsets)
