"""Canonical subspace index.

Lower / upper triangle evaluation section: subspace bit-strings are sorted by their integer
values, so the index of a bit-string is its rank in ascending unsigned order.  Duplicated
samples are removed (Results: "duplicates removed").  Multi-word bit-sets compare as big
unsigned integers (most significant word last in the ``[n][W]`` layout).
"""
import bisect

import numpy as np


def keys_to_ints(keys: np.ndarray) -> list:
    keys = np.asarray(keys, dtype=np.uint64)
    if keys.ndim == 1:
        keys = keys[:, None]
    W = keys.shape[1]
    out = []
    for row in keys.tolist():
        v = 0
        for w in range(W - 1, -1, -1):
            v = (v << 64) | int(row[w])
        out.append(v)
    return out


def ints_to_keys(values, W: int) -> np.ndarray:
    out = np.zeros((len(values), W), dtype=np.uint64)
    for i, v in enumerate(values):
        for w in range(W):
            out[i, w] = (int(v) >> (64 * w)) & 0xFFFFFFFFFFFFFFFF
    return out


def canonical(values) -> list:
    """Sorted distinct Python ints (the index of a value is its position)."""
    return sorted(set(int(v) for v in values))


def canonical_keys(keys: np.ndarray) -> np.ndarray:
    """Sorted distinct ``uint64[n][W]`` rows, ascending as big unsigned integers."""
    keys = np.asarray(keys, dtype=np.uint64)
    if keys.ndim == 1:
        keys = keys[:, None]
    rev = np.ascontiguousarray(keys[:, ::-1])
    uniq = np.unique(rev, axis=0)  # lexicographic, first column most significant
    return np.ascontiguousarray(uniq[:, ::-1])


def index_of(sorted_values: list, v: int) -> int:
    """Rank of ``v`` in ``sorted_values`` or -1."""
    k = bisect.bisect_left(sorted_values, v)
    if k < len(sorted_values) and sorted_values[k] == v:
        return k
    return -1


def is_lower(row: int, col: int) -> bool:
    """Entry ``(row, col)`` lies in the lower triangle iff ``index(col) < index(row)``,
    which under the integer order means ``col < row`` as integers."""
    return col < row
