"""The library's window keys against a per-base construction, on the CPU.

The device kernels compute every sort key with the __host__ __device__
functions of device_common.h (first_key, window_key) from 16-byte text
records.  Here those same functions are compiled host-only and fed records
built in Python from their documented layout; each key must equal the
reading of Section 3.2 taken for this library: the window's bases zero-padded
past the end of the read (first base in the top bits 63..10), the clamped
number of bases left min(remaining, 27) in bits 7..3, and the preceding
symbol (0..3 a base, 4 for '$') in bits 2..0.

Texts hold reads of lengths 0..60 whose starts fall on every offset inside a
record, so every window position, read end and record boundary is covered.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from conftest import ROOT

@pytest.fixture(scope="module")
def wk(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("wk")
    so = str(d / "libwk.so")
    src = os.path.join(ROOT, "tests", "window_keys_host.cpp")
    inc = os.path.join(ROOT, "paper_1401_7457_amd", "csrc")
    subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", inc,
                    src, "-o", so], check=True, capture_output=True)
    L = ctypes.CDLL(so)
    u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
    L.wk_first_key.argtypes = [vp, u64, u64]
    L.wk_first_key.restype = u64
    L.wk_window_key.argtypes = [vp, u64, u64, u32, u32]
    L.wk_window_key.restype = u64
    L.wk_window.restype = u32
    return L


def _records(codes: np.ndarray, read_bounds: list) -> np.ndarray:
    """Text records from the documented layout (one per 16 positions).

    Record w: hi = bases 16w..16w+31 (first base in bits 63..62); lo bits
    63..44 = bases 16w+32..16w+41, bits 43..42 = base 16w-1 (zero for w = 0),
    bit k (k < 42) set when position 16w+k starts a non-empty read or is the
    end of the text B.  Positions past B read as zero; floor(B/16)+2 records.
    """
    B = codes.size
    n_rec = B // 16 + 2
    span = 16 * n_rec + 64
    c = np.zeros(span, dtype=np.uint64)
    c[:B] = codes
    start = np.zeros(span, dtype=bool)
    for a, b in read_bounds:
        if b > a:
            start[a] = True
    start[B] = True
    recs = np.zeros(2 * n_rec, dtype=np.uint64)
    for w in range(n_rec):
        t = 16 * w
        hi = 0
        for k in range(32):
            hi = (hi << 2) | int(c[t + k])
        lo = 0
        for k in range(32, 42):
            lo = (lo << 2) | int(c[t + k])
        lo <<= 44
        if w:
            lo |= int(c[t - 1]) << 42
        for k in range(42):
            if start[t + k]:
                lo |= 1 << k
        recs[2 * w] = hi
        recs[2 * w + 1] = lo
    return recs


def _expected_key(codes, b, q, prev3):
    """(27 bases from q, zero past the read end b) << 10 | min(b - q, 27) << 3 | prev3."""
    clamp = min(b - q, 27)
    key = 0
    for i in range(clamp):
        key |= int(codes[q + i]) << (62 - 2 * i)
    return key | (clamp << 3) | prev3


def _case(rng, n_reads, lead):
    lens = [lead] + [int(x) for x in rng.integers(0, 61, size=n_reads)]
    text = rng.integers(0, 4, size=sum(lens)).astype(np.uint8)
    bounds = []
    a = 0
    for L in lens:
        bounds.append((a, a + L))
        a += L
    return text, bounds


@pytest.mark.parametrize("seed", range(6))
def test_window_keys_match_per_base_construction(wk, seed):
    W = 27
    assert wk.wk_window() == W
    rng = np.random.default_rng(100 + seed)
    checked = 0
    starts_mod16 = set()
    for lead in range(16):  # the first long read pushes later starts to every record offset
        codes, bounds = _case(rng, 12, lead)
        B = codes.size
        recs = _records(codes, bounds)
        ptr = recs.ctypes.data_as(ctypes.c_void_p)
        for a, b in bounds:
            if b > a:
                starts_mod16.add(a % 16)
            for p in range(a, b):
                prev3 = 4 if p == a else int(codes[p - 1])
                got0 = wk.wk_first_key(ptr, B, p)
                assert got0 == _expected_key(codes, b, p, prev3), (seed, lead, a, b, p)
                # window 0 always; window r >= 1 while the read holds 27 r bases from p
                for r in range(0, (b - p) // W + 1):
                    q = p + W * r
                    got = wk.wk_window_key(ptr, B, p, r, prev3)
                    assert got == _expected_key(codes, b, q, prev3), (seed, lead, a, b, p, r)
                    checked += 1
    assert starts_mod16 == set(range(16))
    assert checked > 2000


def test_window_key_of_a_read_ending_at_a_window_edge(wk):
    # a 54-base read: window 2 of its first suffix starts exactly at the read
    # end (no bases left, clamped length 0) and the key is the symbol alone
    codes = np.arange(54, dtype=np.uint8) % 4
    bounds = [(0, 54)]
    recs = _records(codes, bounds)
    ptr = recs.ctypes.data_as(ctypes.c_void_p)
    assert wk.wk_window_key(ptr, 54, 0, 2, 4) == 4
    assert wk.wk_window_key(ptr, 54, 0, 1, 4) == _expected_key(codes, 54, 27, 4)
    assert (wk.wk_first_key(ptr, 54, 0) >> 3) & 31 == 27


def test_empty_reads_do_not_end_a_suffix(wk):
    # empty reads between two reads set no start bit of their own: the first
    # read's suffixes still end where the next non-empty read starts
    codes = np.array([1, 2, 3, 0, 0, 1], dtype=np.uint8)
    bounds = [(0, 3), (3, 3), (3, 3), (3, 6)]
    recs = _records(codes, bounds)
    ptr = recs.ctypes.data_as(ctypes.c_void_p)
    for p in range(3):
        prev3 = 4 if p == 0 else int(codes[p - 1])
        assert wk.wk_first_key(ptr, 6, p) == _expected_key(codes, 3, p, prev3)
    assert wk.wk_first_key(ptr, 6, 3) == _expected_key(codes, 6, 3, 4)
