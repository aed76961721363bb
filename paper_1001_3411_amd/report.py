"""Comparisons between two HOP results on the host (used to report how far a
reduced-precision run lands from the FP64 one).

Both functions take plain numpy arrays in input order.
"""
from __future__ import annotations

import numpy as np

__all__ = ["max_rel_error", "group_change_fraction"]


def max_rel_error(ref: np.ndarray, val: np.ndarray) -> float:
    """max |val - ref| / |ref| over particles with ref != 0."""
    ref = np.asarray(ref, dtype=np.float64)
    val = np.asarray(val, dtype=np.float64)
    nz = ref != 0
    if not nz.any():
        return 0.0
    return float(np.max(np.abs(val[nz] - ref[nz]) / np.abs(ref[nz])))


def group_change_fraction(ref_group: np.ndarray, group: np.ndarray) -> float:
    """Fraction of particles whose group changed between two labellings.

    Groups are matched one to one by shared particles: over all (reference
    group, other group) pairs in decreasing order of shared count (ties to
    the smaller labels), a pair is matched when neither side is matched yet.
    This is the cross-match of halo catalogues that the paper uses to compare
    two runs.  A particle has changed when it is in no group in one
    labelling and in a group in the other, or when its two groups are not
    matched to each other.  The label -1 means no group.
    """
    a = np.asarray(ref_group, dtype=np.int64)
    b = np.asarray(group, dtype=np.int64)
    if a.shape != b.shape:
        raise ValueError("labellings differ in length")
    n = a.size
    if n == 0:
        return 0.0
    both = (a >= 0) & (b >= 0)
    kept = 0
    if both.any():
        pairs = np.stack([a[both], b[both]], axis=1)
        uniq, counts = np.unique(pairs, axis=0, return_counts=True)
        order = np.lexsort((uniq[:, 1], uniq[:, 0], -counts))
        used_a, used_b = set(), set()
        for k in order.tolist():
            ga, gb = int(uniq[k, 0]), int(uniq[k, 1])
            if ga in used_a or gb in used_b:
                continue
            used_a.add(ga)
            used_b.add(gb)
            kept += int(counts[k])
    kept += int(np.count_nonzero((a < 0) & (b < 0)))
    return float(n - kept) / n
