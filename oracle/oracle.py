"""Plain CPU oracle for the multi-string BWT of a read collection.

TEST INFRASTRUCTURE ONLY: the tests, the smoke entry point and the CPU-baseline
leg of the benchmark are the only users.  The product library never imports,
links or runs anything here, and nothing here imports the product library.

The method (Liu, Luo & Lam, Section 2 and Fig. 1): every read r_i becomes
S_i = r_i $_i; all suffixes of all S_i are sorted lexicographically with
$_i < A < C < G < T and $_i < $_j iff i < j; row rho of the BWT is the symbol
preceding the rho-th suffix in its own string, '$' for an offset-0 suffix.

Functions:
  bwt(text, offsets)            -- compiled C comparison sort (cx_oracle.c)
  sorted_suffixes(text, offsets)-- the sorted (read, offset) pairs themselves
  bwt_bruteforce(reads)         -- pure Python, tiny inputs only
  pack(text)                    -- the 2-bit packed input layout, written out
  adjacent_lcp / live_profile   -- ties left after each fixed-width window
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cx_oracle.c")
_LIB = os.path.join(_HERE, "libcx_oracle.so")
_lock = threading.Lock()
_lib = None


def compile_oracle(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the C oracle with gcc into a shared library; returns its path."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-pthread", src, "-o", out]
    subprocess.run(cmd, check=True)
    return out


def load(path: str | None = None):
    """Load (compiling first if needed) the oracle library."""
    global _lib
    with _lock:
        if path is not None:
            return _bind(ctypes.CDLL(path))
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                compile_oracle()
            _lib = _bind(ctypes.CDLL(_LIB))
        return _lib


def _bind(lib):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.cx_oracle_bwt.argtypes = [u8p, u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, u8p, u64p]
    lib.cx_oracle_bwt.restype = ctypes.c_int
    lib.cx_oracle_sorted_suffixes.argtypes = [u8p, u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, u32p]
    lib.cx_oracle_sorted_suffixes.restype = ctypes.c_int
    lib.cx_oracle_validate.argtypes = [u8p, u64p, ctypes.c_uint64, ctypes.c_uint64]
    lib.cx_oracle_validate.restype = ctypes.c_int
    if hasattr(lib, "cx_check_bwt"):
        lib.cx_check_bwt.argtypes = [u8p, u64p, u8p, u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        lib.cx_check_bwt.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_inputs(text, offsets):
    if isinstance(text, (bytes, bytearray, str)):
        text = np.frombuffer(text.encode() if isinstance(text, str) else bytes(text), dtype=np.uint8)
    text = np.ascontiguousarray(text, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if text.size == 0:
        text = np.zeros(1, dtype=np.uint8)[:0]
    return text, offsets


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def bwt(text, offsets, threads: int | None = None, lib=None):
    """BWT rows (uint8 ASCII A/C/G/T/$) and term_pos (uint64 per read).

    text: the reads concatenated (ASCII), offsets: n+1 base offsets.
    """
    text, offsets = _as_inputs(text, offsets)
    n = offsets.size - 1
    nb = int(offsets[-1]) if n >= 0 else 0
    lib = lib or load()
    out = np.empty(nb + n, dtype=np.uint8)
    tp = np.empty(max(n, 0), dtype=np.uint64)
    tbuf = text if text.size else np.zeros(1, dtype=np.uint8)
    st = lib.cx_oracle_bwt(_ptr(tbuf, ctypes.c_uint8), _ptr(offsets, ctypes.c_uint64), n, nb,
                           threads or default_threads(), _ptr(out if out.size else np.zeros(1, np.uint8), ctypes.c_uint8),
                           _ptr(tp if tp.size else np.zeros(1, np.uint64), ctypes.c_uint64))
    if st != 0:
        raise ValueError(f"oracle rejected the input (status {st})")
    return out, tp


def sorted_suffixes(text, offsets, threads: int | None = None, lib=None) -> np.ndarray:
    """(rows, 2) uint32 array of (read, offset) in sorted suffix order."""
    text, offsets = _as_inputs(text, offsets)
    n = offsets.size - 1
    nb = int(offsets[-1])
    lib = lib or load()
    out = np.empty((nb + n, 2), dtype=np.uint32)
    tbuf = text if text.size else np.zeros(1, dtype=np.uint8)
    st = lib.cx_oracle_sorted_suffixes(_ptr(tbuf, ctypes.c_uint8), _ptr(offsets, ctypes.c_uint64), n, nb,
                                       threads or default_threads(),
                                       _ptr(out if out.size else np.zeros(2, np.uint32), ctypes.c_uint32))
    if st != 0:
        raise ValueError(f"oracle rejected the input (status {st})")
    return out


def check_bwt(bwt, term_pos, text, offsets, threads: int | None = None, lib=None) -> int:
    """Counts, bare-terminator rows and the LF walk of every read, in C (0 = all hold).

    1: symbol counts wrong, 2: rows 0..n-1 wrong, 3: an LF walk diverged.
    """
    text, offsets = _as_inputs(text, offsets)
    bwt = np.ascontiguousarray(bwt, dtype=np.uint8)
    tp = np.ascontiguousarray(term_pos, dtype=np.uint64)
    n = offsets.size - 1
    nb = int(offsets[-1])
    lib = lib or load()
    tbuf = text if text.size else np.zeros(1, dtype=np.uint8)
    return int(lib.cx_check_bwt(_ptr(bwt, ctypes.c_uint8), _ptr(tp if tp.size else np.zeros(1, np.uint64), ctypes.c_uint64),
                                _ptr(tbuf, ctypes.c_uint8), _ptr(offsets, ctypes.c_uint64), n, nb,
                                threads or default_threads()))


def bwt_bruteforce(reads: list[str]):
    """Pure-Python BWT for tiny collections, straight from the definition.

    Each suffix becomes a tuple of symbol keys: a base is (1 + rank,) with
    A<C<G<T, the terminator of read i is (0, i), so tuple order is exactly
    the order of Section 2.  Returns (bwt string, term_pos list).
    """
    rank = {"A": 1, "C": 2, "G": 3, "T": 4}
    entries = []
    for i, r in enumerate(reads):
        full = [(rank[c],) for c in r] + [(0, i)]
        for k in range(len(r) + 1):
            entries.append((tuple(full[k:]), i, k))
    entries.sort(key=lambda e: e[0])
    out = []
    term = [0] * len(reads)
    for row, (_, i, k) in enumerate(entries):
        if k == 0:
            out.append("$")
            term[i] = row
        else:
            out.append(reads[i][k - 1])
    return "".join(out), term


def pack(text) -> np.ndarray:
    """The 2-bit packed layout of the library's input, written out.

    A=0, C=1, G=2, T=3; base t of the concatenated reads sits in 64-bit word
    t // 32 at bits [62 - 2 (t % 32), 63 - 2 (t % 32)] (first base in the
    most significant pair).  ceil(n/32) + 1 words: the last word is zero
    padding.
    """
    if isinstance(text, (bytes, bytearray, str)):
        text = np.frombuffer(text.encode() if isinstance(text, str) else bytes(text), dtype=np.uint8)
    text = np.asarray(text, dtype=np.uint8)
    code = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3}
    nb = text.size
    words = np.zeros((nb + 31) // 32 + 1, dtype=np.uint64)
    lut = np.full(256, 255, dtype=np.uint8)
    for ch, v in code.items():
        lut[ch] = v
    codes = lut[text]
    if nb and codes.max() > 3:
        raise ValueError("only A/C/G/T can be packed")
    for t0 in range(0, nb, 32):
        chunk = codes[t0:t0 + 32].astype(np.uint64)
        shifts = (62 - 2 * np.arange(chunk.size)).astype(np.uint64)
        words[t0 // 32] = np.bitwise_or.reduce(chunk << shifts) if chunk.size else 0
    return words


def adjacent_lcp(text, offsets, order: np.ndarray) -> np.ndarray:
    """Bases shared by each sorted suffix and the one before it (row 0: 0).

    `order` is the (rows, 2) array of (read, offset) from sorted_suffixes.
    Terminators are all distinct (Section 2), so a common prefix never
    extends past either suffix's last base.
    """
    text, offsets = _as_inputs(text, offsets)
    order = np.asarray(order, dtype=np.int64)
    rows = order.shape[0]
    lcp = np.zeros(rows, dtype=np.int64)
    if rows < 2:
        return lcp
    start = offsets[order[:, 0]].astype(np.int64) + order[:, 1]
    rem = (offsets[order[:, 0] + 1] - offsets[order[:, 0]]).astype(np.int64) - order[:, 1]
    a, b = start[:-1], start[1:]
    cand = np.nonzero(np.minimum(rem[:-1], rem[1:]) > 0)[0]
    k = 0
    while cand.size:
        same = text[a[cand] + k] == text[b[cand] + k]
        cand = cand[same]
        lcp[cand + 1] += 1
        k += 1
        cand = cand[np.minimum(rem[cand], rem[cand + 1]) > k]
    return lcp


def live_profile(text, offsets, width: int, order: np.ndarray | None = None) -> list[int]:
    """Suffixes still tied after each window of `width` bases (Section 3.2).

    Sorting by successive fixed-width windows leaves a suffix undecided after
    r windows exactly when some other suffix shares its first r*width bases,
    which in sorted order means a neighbour with a common prefix of at least
    r*width bases.  Entry r-1 of the result is that count for r = 1, 2, ...
    up to the last nonzero one; its sum is the number of next-window loads a
    schedule that refines only tied suffixes makes.
    """
    if order is None:
        order = sorted_suffixes(text, offsets)
    lcp = adjacent_lcp(text, offsets, order)
    best = lcp.copy()
    if best.size > 1:
        best[:-1] = np.maximum(best[:-1], lcp[1:])
    out = []
    r = 1
    while True:
        c = int(np.count_nonzero(best >= r * width))
        if c == 0:
            return out
        out.append(c)
        r += 1
