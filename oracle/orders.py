"""Orders of signed and IEEE-754 keys for the oracle -- TEST INFRASTRUCTURE.

The paper's method sorts bit strings; it applies to any data type whose
encoding is made to order it (section "The Other Universal Property").  The
library reads signed and floating-point keys through an order-preserving
unsigned view.  This module states the target orders directly, by value,
with no bit flipping, so that the two can be checked against each other:

* signed: two's-complement integers in numeric order;
* float: the IEEE-754 total order: -NaN < -inf < negative numbers < -0 <
  +0 < positive numbers < +inf < +NaN, NaNs of one sign ordered by their
  payload bits (larger payload further from zero).

Each key is mapped to an integer whose numeric order is that order, and the
result is the stable sort (equal keys keep input order) by that integer.
"""
from __future__ import annotations

import numpy as np

UNSIGNED, SIGNED, FLOAT = 0, 1, 2


def rank_value(keys: np.ndarray, kind: int) -> np.ndarray:
    """An integer per key whose numeric order is the key order of `kind`.
    keys: uint32 or uint64 bit patterns."""
    width = keys.dtype.itemsize * 8
    if keys.dtype not in (np.uint32, np.uint64):
        raise ValueError("keys must be uint32 or uint64 bit patterns")
    if kind == UNSIGNED:
        return keys.astype(object) if width == 64 else keys.astype(np.int64)
    if kind == SIGNED:
        return keys.view(np.int32 if width == 32 else np.int64).astype(np.int64)
    if kind == FLOAT:
        # sign and magnitude: a negative key is placed below every
        # non-negative one, further down the larger its magnitude
        mag_mask = keys.dtype.type((1 << (width - 1)) - 1)
        mag = (keys & mag_mask).astype(np.int64)          # < 2^(width-1): fits
        neg = (keys >> keys.dtype.type(width - 1)) != 0
        return np.where(neg, -mag - 1, mag)              # -mag - 1 >= -2^63
    raise ValueError("kind must be 0, 1 or 2")


def stable_order(keys: np.ndarray, kind: int) -> np.ndarray:
    """The stable sorting permutation (0-based, int64) of `keys` under `kind`."""
    v = rank_value(keys, kind)
    if v.dtype == object:
        # Python's sort is stable: equal values keep input order
        return np.array(sorted(range(keys.shape[0]), key=v.__getitem__), dtype=np.int64)
    return np.argsort(v, kind="stable")


def sort(keys: np.ndarray, payload: np.ndarray | None, kind: int):
    """(sorted keys, payload carried with them) under the order of `kind`."""
    p = stable_order(keys, kind)
    return keys[p], (None if payload is None else payload[p])


def sort_segmented(keys: np.ndarray, seg_offsets: np.ndarray, payload: np.ndarray | None, kind: int):
    """Each segment [off[s], off[s+1]) sorted on its own under `kind`."""
    ko = keys.copy()
    po = None if payload is None else payload.copy()
    off = np.asarray(seg_offsets, dtype=np.int64)
    for s in range(off.shape[0] - 1):
        a, b = int(off[s]), int(off[s + 1])
        if b - a > 1:
            p = stable_order(keys[a:b], kind)
            ko[a:b] = keys[a:b][p]
            if po is not None:
                po[a:b] = payload[a:b][p]
    return ko, po
