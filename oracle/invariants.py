"""Properties every multi-string BWT satisfies, checkable at any size.

TEST INFRASTRUCTURE ONLY (see oracle.py).  These hold for the BWT of Section 2
of Liu, Luo & Lam whatever the input, so they check the oracle on its own and
check large device outputs where a full oracle run would be too slow.

  check_counts      -- the BWT is a permutation of the input bases plus one
                       '$' per read, and term_pos is exactly the set of '$' rows
  check_dollar_rows -- rows 0..n-1 are the bare terminators $_0 < ... < $_{n-1},
                       so row i holds the last base of read i ('$' if empty)
  lf_reconstruct    -- the LF walk (C array + occurrence counts) from row i
                       spells read i backwards and ends at term_pos[i]
"""
from __future__ import annotations

import numpy as np

SYMBOLS = np.frombuffer(b"$ACGT", dtype=np.uint8)


def _codes(bwt: np.ndarray) -> np.ndarray:
    lut = np.full(256, 255, dtype=np.uint8)
    for v, ch in enumerate(b"$ACGT"):
        lut[ch] = v
    c = lut[np.asarray(bwt, dtype=np.uint8)]
    if c.size and c.max() > 4:
        raise AssertionError("BWT holds a symbol outside $ACGT")
    return c


def check_counts(bwt, term_pos, text, offsets) -> None:
    bwt = np.asarray(bwt, dtype=np.uint8)
    text = np.asarray(text, dtype=np.uint8)
    n = len(offsets) - 1
    assert bwt.size == text.size + n, "BWT length must be bases + reads"
    got = np.bincount(_codes(bwt), minlength=5)
    want = np.bincount(_codes(text), minlength=5) if text.size else np.zeros(5, np.int64)
    want = want.copy()
    want[0] += n
    assert np.array_equal(got, want), f"symbol counts differ: {got} vs {want}"
    dollar_rows = np.flatnonzero(bwt == ord("$"))
    tp = np.sort(np.asarray(term_pos, dtype=np.int64))
    assert np.array_equal(tp, dollar_rows), "term_pos is not the set of '$' rows"


def check_dollar_rows(bwt, text, offsets) -> None:
    bwt = np.asarray(bwt, dtype=np.uint8)
    text = np.asarray(text, dtype=np.uint8)
    off = np.asarray(offsets, dtype=np.int64)
    n = off.size - 1
    lens = off[1:] - off[:-1]
    want = np.full(n, ord("$"), dtype=np.uint8)
    nz = lens > 0
    want[nz] = text[off[1:][nz] - 1]
    assert np.array_equal(bwt[:n], want), "rows 0..n-1 must be the bare terminators in read order"


def lf_reconstruct(bwt, term_pos, text, offsets, reads: np.ndarray | None = None) -> None:
    """LF-walk every (or every listed) read and compare with the input.

    C[c] = number of symbols smaller than c (all '$' count below A);
    LF(rho) = C[b] + #{rho' < rho : bwt[rho'] = b} for b = bwt[rho] != '$'.
    Row i is the suffix $_i, so walking LF from row i reads r_i backwards and
    stops on the row whose symbol is '$', which is term_pos[i].
    """
    bwt = np.asarray(bwt, dtype=np.uint8)
    codes = _codes(bwt).astype(np.int64)
    text = np.asarray(text, dtype=np.uint8)
    off = np.asarray(offsets, dtype=np.int64)
    tp = np.asarray(term_pos, dtype=np.int64)
    n = off.size - 1
    counts = np.bincount(codes, minlength=5)
    C = np.concatenate([[0], np.cumsum(counts)[:-1]])
    # occ_before[rho] = #{rho' < rho : codes[rho'] == codes[rho]}
    occ_before = np.empty(codes.size, dtype=np.int64)
    for c in range(5):
        idx = np.flatnonzero(codes == c)
        occ_before[idx] = np.arange(idx.size)
    lf = C[codes] + occ_before
    which = np.arange(n) if reads is None else np.asarray(reads, dtype=np.int64)
    # walk all selected reads in lock-step (vectorised over reads)
    rows = which.copy()
    lens = off[which + 1] - off[which]
    maxlen = int(lens.max()) if lens.size else 0
    for step in range(maxlen + 1):
        live = lens >= step
        if not live.any():
            break
        r = rows[live]
        sym = bwt[r]
        pos = off[which[live] + 1] - 1 - step  # base expected before this suffix
        expect_dollar = step == lens[live]
        exp = np.where(expect_dollar, ord("$"), text[np.clip(pos, 0, max(text.size - 1, 0))] if text.size else ord("$"))
        assert np.array_equal(sym, exp.astype(np.uint8)), f"LF walk diverged at step {step}"
        ended = expect_dollar
        assert np.array_equal(r[ended], tp[which[live][ended]]), "LF walk did not end at term_pos"
        rows[live] = np.where(ended, r, lf[r])
