"""Row fingerprints of neighbour lists (test helper).

Word-wise FNV-1a: h = 0xcbf29ce484222325, then for each 32-bit entry
h = (h xor entry) * 0x100000001b3 mod 2^64.  Written here from the published
FNV-1a definition, independently of the oracle's C version, so that lists
too long to keep for every particle can be compared row by row.
"""
import numpy as np

_BASIS = np.uint64(0xCBF29CE484222325)
_PRIME = np.uint64(0x100000001B3)


def row_fnv1a(nbr, k=None):
    """uint64 fingerprint of each row of an int32 [n][>=k] array."""
    a = np.asarray(nbr)
    k = a.shape[1] if k is None else k
    h = np.full(a.shape[0], _BASIS, dtype=np.uint64)
    with np.errstate(over="ignore"):
        for t in range(k):
            h ^= a[:, t].astype(np.int32).view(np.uint32).astype(np.uint64)
            h *= _PRIME
    return h
