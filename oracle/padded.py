"""Reference of the padded CMRS of Sec. 6.7 (TEST INFRASTRUCTURE ONLY).

Only ``tests/`` may use it.  Sec. 6.7 keeps M = 8 copies of a strip's row
sums per warp (lane l adds into copy l mod M) and makes that safe by
arranging every strip in steps of W = 64 entries where each row contributes
at most M entries, stored contiguously, padding strips with explicit zeros
to whole steps.  The paper states these constraints but no arrangement
order; the reading used by the library (and written out here, in plain
Python, one strip and one chunk at a time) is:

  chunk after chunk, every row of the strip with entries left offers
  t = min(8, entries left) of them, in CSR order; rows with more entries left
  come first, ties by lower row; the offers fill the 64 slots in that order
  (the last one cut to the space left); the slots after them are padding,
  stored as RowInStrip = height, column 0, value +0.

``check_constraints`` verifies the paper's conditions on any arrangement,
independently of the order, and that the stored entries are exactly the
CSR's.  Parity of this function with the printed constraints: see
tests/test_padded_cpu.py.
"""
from __future__ import annotations

import numpy as np

M = 8
W = 64


def padded_bits(height: int) -> int:
    """Width of the RowInStrip field: values 0 .. height (padding = height)."""
    b = 0
    while (1 << b) < height + 1:
        b += 1
    return max(4, b)


def arrange(row_ptr, col_ind, val, height):
    """(strip_ptr, word, val) of the padded matrix, val as given (any dtype)."""
    row_ptr = [int(v) for v in row_ptr]
    rows = len(row_ptr) - 1
    bits = padded_bits(height)
    strips = (rows + height - 1) // height
    strip_ptr = [0]
    words, vals = [], []
    zero = np.zeros(1, dtype=np.asarray(val).dtype)[0]
    for s in range(strips):
        r0 = s * height
        nr = min(height, rows - r0)
        start = [row_ptr[r0 + r] for r in range(nr)]
        left = [row_ptr[r0 + r + 1] - row_ptr[r0 + r] for r in range(nr)]
        used = [0] * nr
        while any(left):
            order = sorted(range(nr), key=lambda r: (-left[r], r))
            slots = []
            for r in order:
                t = min(M, left[r], W - len(slots))
                for q in range(t):
                    slots.append((r, start[r] + used[r] + q))
                used[r] += t
                left[r] -= t
            for r, k in slots:
                words.append((int(col_ind[k]) << bits) | r)
                vals.append(val[k])
            for _ in range(W - len(slots)):
                words.append(height)
                vals.append(zero)
        strip_ptr.append(len(words))
    return (np.asarray(strip_ptr, dtype=np.int64), np.asarray(words, dtype=np.uint32),
            np.asarray(vals, dtype=np.asarray(val).dtype))


def check_constraints(row_ptr, col_ind, val, height, strip_ptr, word, pval):
    """Assert the Sec. 6.7 conditions on a padded matrix: strips hold whole
    chunks of 64; in every chunk each row's entries are one contiguous run of
    at most 8; padding entries are (row = height, value 0); the non-padding
    entries of strip s are exactly the CSR entries of its rows, each row's in
    CSR order."""
    bits = padded_bits(height)
    mask = (1 << bits) - 1
    rows = len(row_ptr) - 1
    strips = (rows + height - 1) // height
    assert len(strip_ptr) == strips + 1 and strip_ptr[0] == 0 and strip_ptr[-1] == len(word)
    word = np.asarray(word, dtype=np.uint32)
    for s in range(strips):
        p0, p1 = int(strip_ptr[s]), int(strip_ptr[s + 1])
        assert (p1 - p0) % W == 0
        got = {}
        for c in range(p0, p1, W):
            rr = (word[c:c + W] & mask).astype(np.int64)
            seen = set()
            prev = -1
            run = 0
            for q in range(W):
                r = int(rr[q])
                if r == height:
                    assert pval[c + q] == 0 and int(word[c + q]) == height
                    prev = -1
                    continue
                assert 0 <= r < height
                if r != prev:
                    assert r not in seen, f"row {r} twice in chunk {c}"
                    seen.add(r)
                    run = 0
                run += 1
                assert run <= M
                prev = r
                got.setdefault(r, []).append((int(word[c + q] >> bits), pval[c + q]))
        for r in range(min(height, rows - s * height)):
            a, b = int(row_ptr[s * height + r]), int(row_ptr[s * height + r + 1])
            want = [(int(col_ind[k]), val[k]) for k in range(a, b)]
            have = got.get(r, [])
            assert len(have) == len(want)
            for (c1, v1), (c2, v2) in zip(have, want):
                assert c1 == c2 and np.asarray(v1).tobytes() == np.asarray(v2).tobytes()


def spmv_by_definition(strip_ptr, word, pval, rows, height, x):
    """y from the padded arrays: every non-padding entry adds val * x[col] to
    row strip * height + RowInStrip (fp64, entries in storage order)."""
    bits = padded_bits(height)
    mask = (1 << bits) - 1
    y = np.zeros(rows)
    for s in range(len(strip_ptr) - 1):
        for k in range(int(strip_ptr[s]), int(strip_ptr[s + 1])):
            r = int(word[k]) & mask
            if r == height:
                continue
            y[s * height + r] += float(pval[k]) * float(x[int(word[k]) >> bits])
    return y
