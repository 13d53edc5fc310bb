"""Several sources per frame (the paper leaves multiple-source localisation
to future work, Section 5).  Test infrastructure only: see the package
docstring.

Reading adopted: the n peaks of a frame's powers y over the grid are taken
greedily.  Peak p is the largest y among the directions whose unit vector
is farther than the separation from every earlier peak (dot product below
cos_sep) and is not itself an earlier peak, ties going to the lowest index;
when no direction is left, the peak is -1 with value -inf.  The dot products and comparisons are done in
float32, each product rounded before the sums ((x x' + y y') + z z'), the
precision in which the GPU takes the same decisions."""
from __future__ import annotations

import numpy as np


def peaks(y: np.ndarray, dirs: np.ndarray, n: int, cos_sep: float):
    """y [F, Q] (float32), dirs [Q, 3] unit vectors -> idx [F, n] int32,
    val [F, n] float32."""
    y = np.asarray(y, dtype=np.float32)
    d = np.asarray(dirs, dtype=np.float32)
    cs = np.float32(cos_sep)
    F, Q = y.shape
    idx = np.full((F, n), -1, dtype=np.int32)
    val = np.full((F, n), -np.inf, dtype=np.float32)
    for f in range(F):
        free = np.ones(Q, dtype=bool)
        for p in range(n):
            cand = np.flatnonzero(free & (y[f] == y[f]))   # NaN never counts
            if cand.size == 0:
                break
            q = int(cand[np.argmax(y[f, cand])])             # first of the maxima
            idx[f, p], val[f, p] = q, y[f, q]
            dot = (d[:, 0] * d[q, 0] + d[:, 1] * d[q, 1]) + d[:, 2] * d[q, 2]
            free &= ~(dot >= cs)
            free[q] = False                                  # the peak itself, whatever cos_sep is
    return idx, val
