"""Plain definition of the sort result -- TEST INFRASTRUCTURE ONLY.

Section "Sorting Formalism" defines sorting as finding a permutation p with
K_p(1) <= K_p(2) <= ... <= K_p(N).  Equal keys admit several such p; the
stable one keeps equal keys in input order, i.e. it orders the pairs
(bit string of key i, i) lexicographically.  The bit string of a key is its
encoding (section "The Other Universal Property"): the big-endian bytes of an
unsigned integer, or the bytes of a string as stored.

This is that definition written out with Python's sort over (bytes, index)
pairs.  It shares no code with the recursive oracle in ``binar_ref.c``.
"""
from __future__ import annotations

import numpy as np


def bit_string(keys: np.ndarray, i: int) -> bytes:
    """Encoding of key i, most significant bit first."""
    if keys.ndim == 2:
        return bytes(keys[i].tolist())
    width = keys.dtype.itemsize
    return int(keys[i]).to_bytes(width, "big")


def stable_permutation(keys: np.ndarray) -> list[int]:
    """The unique stable sorting permutation p (0-based)."""
    n = keys.shape[0]
    return sorted(range(n), key=lambda i: (bit_string(keys, i), i))


def sort(keys: np.ndarray, payload: np.ndarray | None = None):
    """(keys, payload) rearranged by the stable sorting permutation."""
    p = np.asarray(stable_permutation(keys), dtype=np.int64)
    out_k = keys[p] if keys.shape[0] else keys.copy()
    out_p = None if payload is None else np.asarray(payload)[p]
    return out_k, out_p


def stable_rank_u(keys: np.ndarray, j: int) -> int:
    """Output position of input element j under the stable sort of unsigned
    integer keys: keys strictly smaller, plus equal keys earlier in the
    input.  One output at a time, for spot checks of very large sorts."""
    kj = keys[j]
    return int(np.count_nonzero(keys < kj)) + int(np.count_nonzero(keys[:j] == kj))


def stable_rank_bytes(keys: np.ndarray, j: int) -> int:
    """Output position of input string j (a row of a uint8 (n, w) array of
    fixed-length byte strings) under the stable sort: rows that are smaller
    at their first byte differing from row j, plus rows equal to row j that
    come earlier in the input.  One output at a time, for spot checks of
    large sorts."""
    kj = keys[j]
    ne = keys != kj[None, :]
    differs = ne.any(axis=1)
    first = ne.argmax(axis=1)
    rows = np.arange(keys.shape[0])
    smaller = differs & (keys[rows, first] < kj[first])
    return int(np.count_nonzero(smaller)) + int(np.count_nonzero(~differs[:j]))
