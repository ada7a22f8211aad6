"""Geometric nested-dissection ordering of the gauged global system (oracle).

The oracle's result is the plain solution of the gauged global system
W_g a = f_g (Sec. 2.2, implicit Euler system, restricted to the kept edges of
the split of Sec. 3).  Any symmetric permutation P gives the same solution,
a = P^T (P W_g P^T)^{-1} P f_g, so the ordering only decides how much the
sparse factor fills in, and therefore whether the full-size systems can be
factored on one CPU at all.  It takes no part in the arithmetic of the
result.

The ordering is recursive coordinate bisection of the matrix graph: each
unknown sits at the midpoint of its control-grid edge; a set larger than
``leaf`` is split at the median of its longest extent; the unknowns of the
lower half that are coupled (a structural nonzero of W_g) to the upper half
form the separator; the two remaining halves are ordered first, each by the
same rule, and the separator last.  Removing the separator leaves no
nonzero between the halves (``splits`` records each split so that a test
can check this), which is what confines the fill to the separator blocks.

Test infrastructure: only ``tests/``, the smoke check and the CPU baseline
of the benchmark use anything under ``oracle/``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def edge_midpoints(grid, edges):
    """Midpoints of global edges in control-index coordinates, shape (n, 3)."""
    d, I, J, K = grid.edge_decode(edges)
    xyz = np.stack([I, J, K], axis=1).astype(np.float64)
    xyz[np.arange(len(xyz)), d] += 0.5
    return xyz


def nested_dissection(A, xyz, leaf=64, splits=None):
    """Permutation of the unknowns of A: perm[new position] = old index.

    A is a structurally symmetric sparse matrix, xyz the (n, 3) coordinates
    of its unknowns.  If ``splits`` is a list, every split is appended to it
    as (lower half, upper half, separator), index arrays into A.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    indptr, indices = A.indptr, A.indices
    upper = np.zeros(n, dtype=bool)
    perm = []

    def rec(idx):
        if len(idx) <= leaf:
            perm.append(idx)
            return
        pts = xyz[idx]
        ext = pts.max(axis=0) - pts.min(axis=0)
        ax = int(np.argmax(ext))
        med = np.median(pts[:, ax])
        low = pts[:, ax] < med
        if low.all() or not low.any():
            low = pts[:, ax] <= med
        if low.all() or not low.any():
            perm.append(idx)
            return
        lo, hi = idx[low], idx[~low]
        # separator: unknowns of the lower half with a neighbour in the upper
        upper[hi] = True
        starts, cnt = indptr[lo], indptr[lo + 1] - indptr[lo]
        first = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        pos = np.repeat(starts - first, cnt) + np.arange(int(cnt.sum()))
        owner = np.repeat(np.arange(len(lo)), cnt)
        touched = np.zeros(len(lo), dtype=bool)
        touched[owner[upper[indices[pos]]]] = True
        upper[hi] = False
        sep, lo_rest = lo[touched], lo[~touched]
        if splits is not None:
            splits.append((lo_rest, hi, sep))
        rec(lo_rest)
        rec(hi)
        perm.append(sep)

    rec(np.arange(n))
    return np.concatenate(perm) if perm else np.zeros(0, dtype=np.int64)
