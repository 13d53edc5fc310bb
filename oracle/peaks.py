"""Several sources per frame (the paper leaves multiple-source localisation
to future work, Section 5).  Test infrastructure only: see the package
docstring.

Reading adopted: the n peaks of a frame's powers y over the grid are taken
greedily.  Peak p is the largest y among the directions that are not an
earlier peak and whose unit vector is farther than the separation from every
earlier peak, i.e. whose dot product with it is below cos_sep (a dot product
equal to cos_sep is too close).  Ties go to the lowest index; NaN powers
never count; when no direction is left the peak is -1 with value -inf.

The dot products are taken in FP64 from the directions as given.  A library
that forms them in a lower precision can decide differently only where a
dot product lies within its rounding error of cos_sep, so the oracle also
reports, per frame, how many leading peaks were chosen before any such
undecided comparison (|dot - cos_sep| <= band) could have changed the free
set: those peaks are unique, the later ones are checked for validity
instead (``valid_peaks``)."""
from __future__ import annotations

import numpy as np


def peaks(y: np.ndarray, dirs: np.ndarray, n: int, cos_sep: float, band: float = 0.0):
    """y [F, Q] powers, dirs [Q, 3] unit vectors -> (idx [F, n] int64,
    val [F, n] of y's dtype, decided [F] int64).

    decided[f] is the number of leading peaks of frame f that no comparison
    within ``band`` of cos_sep precedes (n when there was none, and always
    n for band = 0)."""
    y = np.asarray(y)
    d = np.asarray(dirs, dtype=np.float64)
    cs = float(cos_sep)
    F, Q = y.shape
    idx = np.full((F, n), -1, dtype=np.int64)
    val = np.full((F, n), -np.inf, dtype=y.dtype if y.dtype.kind == "f" else np.float64)
    decided = np.full(F, n, dtype=np.int64)
    valid = y == y                                         # NaN never counts
    for f in range(F):
        free = valid[f].copy()
        for p in range(n):
            cand = np.flatnonzero(free)
            if cand.size == 0:
                break
            q = int(cand[np.argmax(y[f, cand])])               # first of the maxima
            idx[f, p], val[f, p] = q, y[f, q]
            dot = d @ d[q]
            if band > 0 and decided[f] == n and p + 1 < n and np.any(free & (np.abs(dot - cs) <= band)):
                decided[f] = p + 1
            free &= ~(dot >= cs)
            free[q] = False                                  # the peak itself, whatever cos_sep is
    return idx, val, decided


def valid_peaks(y: np.ndarray, dirs: np.ndarray, cos_sep: float, band: float, idx: np.ndarray) -> np.ndarray:
    """Checks, per frame, that the peaks idx [F, n] are a greedy choice that
    some rounding of the comparisons within ``band`` of cos_sep allows:
    every peak is a non-NaN direction not chosen before, at least
    cos_sep - band away from every earlier peak, no smaller than any direction
    that is clearly free (dot below cos_sep - band with every earlier peak),
    the lowest index among clearly free directions of equal power, and -1
    only when no direction is clearly free.  Returns a bool [F]."""
    y = np.asarray(y, dtype=np.float64)
    d = np.asarray(dirs, dtype=np.float64)
    F, Q = y.shape
    ok = np.ones(F, dtype=bool)
    nan = y != y
    for f in range(F):
        surely = ~nan[f]               # free under every rounding
        maybe = ~nan[f]                # free under some rounding
        for p in range(idx.shape[1]):
            q = int(idx[f, p])
            if q < 0:
                if np.any(surely):
                    ok[f] = False
                # once empty, stays empty
                if np.any(idx[f, p:] >= 0):
                    ok[f] = False
                break
            if not maybe[q]:
                ok[f] = False
                break
            if np.any(surely):
                best = np.max(y[f, surely])
                if y[f, q] < best:
                    ok[f] = False
                    break
                if y[f, q] == best:
                    first = int(np.flatnonzero(surely & (y[f] == best))[0])
                    if q > first:
                        ok[f] = False
                        break
            dot = d @ d[q]
            surely &= dot < cos_sep - band
            maybe &= dot < cos_sep + band
            surely[q] = maybe[q] = False
    return ok
