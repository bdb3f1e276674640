"""Pure-Python brute force for tiny matrices (TEST INFRASTRUCTURE ONLY).

These are written independently of ``cmrs_oracle.c`` and serve to pin it:
  * ``dense_from_coo`` / ``dense_matvec`` follow y = A x on a dense array
    (Sec. 2.1), with repeated (row, col) entries adding (COO, Sec. 2.3);
  * ``exact_matvec`` computes y = A x in exact rational arithmetic
    (``fractions.Fraction``), the value every floating-point result is
    measured against;
  * ``cmrs_by_definition`` builds the CMRS arrays of Sec. 3 literally, one
    entry at a time, from the COO triplets, including the in-strip reorder of
    Sec. 4 (by column, then RowInStrip, ties in CRS order).
Only for cases of a few hundred entries.
"""
from __future__ import annotations

from fractions import Fraction


def coo_from_csr(row_ptr, col_ind, val):
    out = []
    for i in range(len(row_ptr) - 1):
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            out.append((i, int(col_ind[k]), val[k]))
    return out


def dense_from_coo(rows, cols, coo):
    a = [[0.0] * cols for _ in range(rows)]
    for i, j, v in coo:
        a[i][j] += float(v)
    return a


def dense_matvec(a, x):
    y = []
    for row in a:
        s = 0.0
        for aij, xj in zip(row, x):
            s = s + aij * float(xj)
        y.append(s)
    return y


def exact_matvec(rows, coo, x):
    """y = A x with every product and sum exact (rationals)."""
    y = [Fraction(0)] * rows
    for i, j, v in coo:
        y[i] += Fraction(float(v)) * Fraction(float(x[j]))
    return y


def cmrs_by_definition(rows, height, coo_in_crs_order, sorted_=False):
    """Returns (strip_ptr, col_ind, row_in_strip, val) as Python lists.

    Strip j holds rows j*height .. j*height+height-1 (Sec. 3); StripPtr[j] is
    the index of its first entry, StripPtr[strips] = nnz; RowInStrip is the row
    number modulo height.
    """
    strips = -(-rows // height)
    by_strip = [[] for _ in range(strips)]
    for pos, (i, j, v) in enumerate(coo_in_crs_order):
        by_strip[i // height].append((j, i % height, pos, v))
    strip_ptr = [0]
    cols, ris, vals = [], [], []
    for items in by_strip:
        if sorted_:
            items = sorted(items, key=lambda t: (t[0], t[1], t[2]))
        for j, r, _pos, v in items:
            cols.append(j)
            ris.append(r)
            vals.append(v)
        strip_ptr.append(len(cols))
    return strip_ptr, cols, ris, vals


def exact_absmv(rows, coo, x):
    """(|A||x|)_i = sum over the entries of row i of |a_ij| |x_j|, exact
    (rationals).  The scale of the componentwise error bound; repeated
    (row, col) entries each contribute their own term, as each is a separate
    product in y = A x."""
    out = [Fraction(0)] * rows
    for i, j, v in coo:
        out[i] += abs(Fraction(float(v))) * abs(Fraction(float(x[j])))
    return out
