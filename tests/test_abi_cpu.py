"""The C ABI without a GPU: symbols, workspace sizing and host-side validation.

Every call here returns before any HIP runtime call (argument checks come
first), so it runs on a machine without a GPU.
"""
import ctypes
import os
import re

import pytest

from conftest import ROOT
from paper_1401_7457_amd import cxbwt

HEADER = os.path.join(ROOT, "include", "cxbwt.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cxbwt_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert set(names) == set(cxbwt.ABI_FUNCTIONS)
    L = cxbwt.lib()
    for name in names:
        assert hasattr(L, name), name


def test_packed_words():
    assert cxbwt.packed_words(0) == 1
    assert cxbwt.packed_words(1) == 2
    assert cxbwt.packed_words(32) == 2
    assert cxbwt.packed_words(33) == 3


def test_workspace_bytes_scale_and_limits():
    small = cxbwt.workspace_bytes(10, 1000, 100)
    big = cxbwt.workspace_bytes(4_000_000, 400_000_000, 100)
    assert small > 24 * 1000
    assert 24 * 400_000_000 <= big <= 28 * 400_000_000
    assert cxbwt.workspace_bytes(0, 10, 10) == 0            # no reads
    assert cxbwt.workspace_bytes(1, 1 << 32, 10) == 0       # above 32-bit handles
    assert cxbwt.workspace_bytes(1, 10, 70000) == 0         # read length bound


def test_build_argument_validation_needs_no_gpu():
    L = cxbwt.lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    args = lambda **kw: [kw.get("packed", fake), kw.get("offsets", fake), kw.get("n", 3), kw.get("nb", 12),
                         kw.get("maxlen", 4), kw.get("bwt", fake), kw.get("term", fake), kw.get("ws", fake),
                         kw.get("wsb", 1 << 40), kw.get("opts"), null]
    assert L.cxbwt_build(*args(packed=null)) == cxbwt.EINVAL
    assert L.cxbwt_build(*args(bwt=null)) == cxbwt.EINVAL
    assert L.cxbwt_build(*args(term=null)) == cxbwt.EINVAL
    assert L.cxbwt_build(*args(ws=null)) == cxbwt.EINVAL
    assert L.cxbwt_build(*args(n=0)) == cxbwt.EINVAL
    assert L.cxbwt_build(*args(nb=1 << 32)) == cxbwt.ERANGE
    assert L.cxbwt_build(*args(maxlen=1 << 20)) == cxbwt.ERANGE
    assert L.cxbwt_build(*args(wsb=10)) == cxbwt.ENOMEM
    assert L.cxbwt_build(*args(ws=ctypes.c_void_p(0x1001))) == cxbwt.EINVAL  # misaligned workspace
    # options the library does not hold are refused before any HIP call (the
    # buffers here are fake, so a call that got further would not return)
    t, c = cxbwt.TUNING_CHOICES[0]
    assert L.cxbwt_build(*args(opts=ctypes.byref(cxbwt.Opts(t, c + 1, cxbwt.SCHEDULE_MSD, 0)))) == cxbwt.EINVAL
    assert L.cxbwt_build(*args(opts=ctypes.byref(cxbwt.Opts(t, c, 2, 0)))) == cxbwt.EINVAL


def test_noalloc_argument_validation_needs_no_gpu():
    """cxbwt_build_noalloc checks its arguments and its array's size before any HIP call."""
    L = cxbwt.lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    args = lambda **kw: [kw.get("packed", fake), kw.get("offsets", fake), kw.get("n", 3), kw.get("nb", 12),
                         kw.get("maxlen", 4), kw.get("bwt", fake), kw.get("term", fake), null]
    assert L.cxbwt_build_noalloc(*args(packed=null)) == cxbwt.EINVAL
    assert L.cxbwt_build_noalloc(*args(offsets=null)) == cxbwt.EINVAL
    assert L.cxbwt_build_noalloc(*args(bwt=null)) == cxbwt.EINVAL
    assert L.cxbwt_build_noalloc(*args(term=null)) == cxbwt.EINVAL
    assert L.cxbwt_build_noalloc(*args(n=0)) == cxbwt.EINVAL
    assert L.cxbwt_build_noalloc(*args(nb=1 << 32)) == cxbwt.ERANGE
    # largest input of 100-base reads the array holds, and one read more
    nb = 9_000_000
    assert cxbwt.workspace_bytes(nb // 100, nb, 100) <= cxbwt.NOALLOC_WORKSPACE_BYTES
    big = 10_000_000
    assert cxbwt.workspace_bytes(big // 100, big, 100) > cxbwt.NOALLOC_WORKSPACE_BYTES
    assert L.cxbwt_build_noalloc(*args(n=big // 100, nb=big, maxlen=100)) == cxbwt.ESCRATCH
    assert b"fixed device array" in L.cxbwt_status_str(cxbwt.ESCRATCH)


def test_range_argument_validation_needs_no_gpu():
    """cxbwt_build_ranges checks its arguments before any HIP call."""
    L = cxbwt.lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)

    def call(**kw):
        return L.cxbwt_build_ranges(kw.get("packed", fake), fake, kw.get("n", 3), kw.get("nb", 12), 4,
                                    kw.get("m", 5), kw.get("flags", 0), fake, fake, kw.get("ws", fake),
                                    kw.get("wsb", 1 << 40), null)

    assert call(packed=null) == cxbwt.EINVAL
    assert call(ws=null) == cxbwt.EINVAL
    assert call(n=0) == cxbwt.EINVAL
    assert call(m=0) == cxbwt.EINVAL
    assert call(flags=2) == cxbwt.EINVAL
    assert call(m=1 << 32) == cxbwt.ERANGE                      # a range must fit 32-bit handles
    assert call(nb=(1 << 38) + 1) == cxbwt.ERANGE                # above the wide-position limit
    assert call(wsb=10) == cxbwt.ENOMEM
    assert call(ws=ctypes.c_void_p(0x1001)) == cxbwt.EINVAL      # misaligned workspace
    # above 32-bit positions only in ranges, with 64-bit position tables
    big = 5_000_000_000
    assert cxbwt.workspace_bytes(50_000_000, big, 100) == 0
    narrow = cxbwt.range_workspace_bytes(4_000_000, 400_000_000, 100, 10_000_000)
    wide = cxbwt.range_workspace_bytes(4_000_000, 400_000_000, 100, 10_000_000, wide=True)
    assert wide - narrow >= 8 * 10_000_000
    assert cxbwt.range_workspace_bytes(50_000_000, big, 100, 1_000_000_000) > 0
    assert cxbwt.range_workspace_bytes(50_000_000, big, 100, 0) == 0


def test_range_workspace_is_smaller_and_monotone():
    n, nb = 4_000_000, 400_000_000
    whole = cxbwt.workspace_bytes(n, nb, 100)
    part = cxbwt.range_workspace_bytes(n, nb, 100, 50_000_000)
    assert part < whole / 3
    assert cxbwt.range_workspace_bytes(n, nb, 100, 50_000_000, wide=True) > part
    sizes = [cxbwt.range_workspace_bytes(n, nb, 100, m) for m in (1, 10, 1000, 10 ** 6, 10 ** 8, nb)]
    assert sizes == sorted(sizes)                       # grows with the budget
    assert sizes[0] > nb                                 # text records and ranks stay whole
    assert cxbwt.range_budget_for(n, nb, 100, part) == 50_000_000
    assert cxbwt.range_budget_for(n, nb, 100, 1000) == 0


def test_job_argument_validation_needs_no_gpu():
    """cxbwt_build_start / cxbwt_build_batch_start check their arguments before
    any HIP call (the job pointer is cleared); waiting on NULL is refused."""
    L = cxbwt.lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)

    def start(**kw):
        h = ctypes.c_void_p(0x1234)
        rc = L.cxbwt_build_start(kw.get("packed", fake), fake, kw.get("n", 3), kw.get("nb", 12), 4, fake, fake,
                                 kw.get("ws", fake), kw.get("wsb", 1 << 40), kw.get("opts"), null, ctypes.byref(h))
        return rc, h.value

    assert start(packed=null) == (cxbwt.EINVAL, None)
    assert start(n=0)[0] == cxbwt.EINVAL
    assert start(nb=1 << 32)[0] == cxbwt.ERANGE
    assert start(wsb=10) == (cxbwt.ENOMEM, None)
    assert start(ws=ctypes.c_void_p(0x1001))[0] == cxbwt.EINVAL
    assert L.cxbwt_build_start(fake, fake, 3, 12, 4, fake, fake, fake, 1 << 40, None, null, None) == cxbwt.EINVAL
    # per-call options: an instantiation the library does not hold, or an unknown schedule
    t, c = cxbwt.TUNING_CHOICES[0]
    assert start(opts=ctypes.byref(cxbwt.Opts(t + 1, c, cxbwt.SCHEDULE_MSD, 0))) == (cxbwt.EINVAL, None)
    assert start(opts=ctypes.byref(cxbwt.Opts(t, c, 7, 0))) == (cxbwt.EINVAL, None)
    # with valid options the other checks still apply
    assert start(opts=ctypes.byref(cxbwt.Opts(t, c, cxbwt.SCHEDULE_STRINGWORD, 1)), wsb=10) == (cxbwt.ENOMEM, None)

    def bstart(coll, wsb=1 << 40):
        h = ctypes.c_void_p(0x1234)
        arr = (ctypes.c_uint64 * len(coll))(*coll)
        rc = L.cxbwt_build_batch_start(fake, fake, 4, 40, 10, arr, len(coll) - 1, fake, fake, fake, wsb, None,
                                       null, ctypes.byref(h))
        return rc, h.value

    assert bstart([0, 2, 3]) == (cxbwt.EINVAL, None)
    assert bstart([0, 2, 2, 4])[0] == cxbwt.EINVAL
    assert bstart([0, 2, 4], wsb=10)[0] == cxbwt.ENOMEM
    assert L.cxbwt_job_wait(null, None) == cxbwt.EINVAL
    assert L.cxbwt_job_done(null) == 0


def test_schedule_set_and_get_without_gpu():
    assert cxbwt.get_schedule() == cxbwt.SCHEDULE_MSD
    try:
        cxbwt.set_schedule(cxbwt.SCHEDULE_STRINGWORD)
        assert cxbwt.get_schedule() == cxbwt.SCHEDULE_STRINGWORD
        with pytest.raises(cxbwt.CxbwtError):
            cxbwt.set_schedule(7)
        assert cxbwt.get_schedule() == cxbwt.SCHEDULE_STRINGWORD
    finally:
        cxbwt.set_schedule(cxbwt.SCHEDULE_MSD)


def test_pack_argument_validation_needs_no_gpu():
    L = cxbwt.lib()
    null = ctypes.c_void_p(0)
    assert L.cxbwt_pack(null, 10, ctypes.c_void_p(0x1000), null, null) == cxbwt.EINVAL
    assert L.cxbwt_pack(ctypes.c_void_p(0x1000), 10, null, null, null) == cxbwt.EINVAL
    assert L.cxbwt_pack(ctypes.c_void_p(0x1000), (1 << 38) + 1, ctypes.c_void_p(0x1000), null, null) == cxbwt.ERANGE


def test_status_strings():
    L = cxbwt.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.cxbwt_status_str(code)
    assert b"unknown" in L.cxbwt_status_str(42)


def test_binding_has_no_cpu_fallback(monkeypatch, tmp_path):
    monkeypatch.setattr(cxbwt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(cxbwt, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        cxbwt.lib()


def test_batch_argument_validation_needs_no_gpu():
    L = cxbwt.lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)

    def call(coll, n=4, nb=40, wsb=1 << 40, ws=fake):
        arr = (ctypes.c_uint64 * len(coll))(*coll)
        return L.cxbwt_build_batch(fake, fake, n, nb, 10, arr, len(coll) - 1, fake, fake, ws, wsb, None, null)

    assert call([0, 2, 3]) == cxbwt.EINVAL          # does not end at n_reads
    assert call([1, 2, 4]) == cxbwt.EINVAL          # does not start at 0
    assert call([0, 2, 2, 4]) == cxbwt.EINVAL       # empty collection
    assert call([0, 2, 4], wsb=10) == cxbwt.ENOMEM
    assert call([0, 2, 4], nb=1 << 32) == cxbwt.ERANGE
    assert cxbwt.batch_workspace_bytes(4, 40, 10, 2) >= cxbwt.workspace_bytes(4, 40, 10)
    assert cxbwt.batch_workspace_bytes(4, 40, 10, 0) == 0
    assert cxbwt.batch_workspace_bytes(4, 40, 10, 5) == 0


def test_graph_argument_validation_needs_no_gpu():
    """cxbwt_graph_* reject bad arguments before any HIP call."""
    L = cxbwt.lib()
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)

    def create(coll, n=4, nb=40, wsb=1 << 40, ws=fake, packed=fake, out=True):
        h = ctypes.c_void_p(0x1234)
        arr = (ctypes.c_uint64 * len(coll))(*coll) if coll is not None else None
        ncoll = len(coll) - 1 if coll is not None else 1
        rc = L.cxbwt_graph_create(packed, fake, n, nb, 10, arr, ncoll, fake, fake, ws, wsb, 0, null,
                                  ctypes.byref(h) if out else None)
        return rc, h.value

    rc, h = create([0, 2, 4], packed=null)
    assert rc == cxbwt.EINVAL and h is None       # null input; *out cleared
    assert create([0, 2, 3])[0] == cxbwt.EINVAL   # does not end at n_reads
    assert create([0, 2, 2, 4])[0] == cxbwt.EINVAL  # empty collection
    assert create([0, 2, 4], wsb=10)[0] == cxbwt.ENOMEM
    assert create([0, 2, 4], ws=ctypes.c_void_p(0x1001))[0] == cxbwt.EINVAL  # workspace not 256-aligned
    assert create([0, 2, 4], nb=1 << 32)[0] == cxbwt.ERANGE
    assert create(None, wsb=10)[0] == cxbwt.ENOMEM  # one collection when coll_reads is NULL
    assert create([0, 2, 4], out=False)[0] == cxbwt.EINVAL
    assert L.cxbwt_graph_launch(null, null) == cxbwt.EINVAL
    assert L.cxbwt_graph_finish(null, null) == cxbwt.EINVAL
    L.cxbwt_graph_destroy(null)  # ignored


def test_tuning_choices_set_and_get_without_gpu():
    before = cxbwt.get_tuning()
    assert before == cxbwt.TUNING_CHOICES[0]
    try:
        for ch in cxbwt.TUNING_CHOICES:
            cxbwt.set_tuning(*ch)
            assert cxbwt.get_tuning() == ch
        for bad in ((0, 8), (32, 8), (12, 8), (8, 2), (8, 4), (8, 16), (7, 6), (16, 16)):
            with pytest.raises(cxbwt.CxbwtError):
                cxbwt.set_tuning(*bad)
        assert cxbwt.get_tuning() == cxbwt.TUNING_CHOICES[-1]
    finally:
        cxbwt.set_tuning(*before)


def test_autotune_shape_key_classes():
    from paper_1401_7457_amd import autotune
    a = autotune.shape_key(4_000_000, 400_000_000, 100)
    assert a == autotune.shape_key(4_100_000, 410_000_000, 100)
    assert a != autotune.shape_key(40_000_000, 4_000_000_000, 100)
    assert a != autotune.shape_key(2_000_000, 400_000_000, 250)


def test_ceilings_gather_library_checks_arguments_without_a_gpu():
    """The measurement kernel of bench.py --mode ceilings is built beside the
    library; invalid arguments are refused before any HIP call."""
    path = os.path.join(os.path.dirname(cxbwt.LIB_PATH), "libcxbwt_ceilings.so")
    L = ctypes.CDLL(path)
    f = L.cxbwt_ceiling_gather
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    fake, sink = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert f(None, 1 << 20, 16, 10, 1, sink, None) == -1          # no table
    assert f(fake, 1000, 16, 10, 1, sink, None) == -1             # rows not a power of two
    assert f(fake, 1 << 20, 24, 10, 1, sink, None) == -1          # row size
    assert f(ctypes.c_void_p(0x1008), 1 << 20, 16, 10, 1, sink, None) == -1  # misaligned table
