"""Order of variable-length byte strings for the oracle -- TEST INFRASTRUCTURE.

The plain definition: string i is data[offsets[i]:offsets[i+1]]; strings are
ordered by their bytes (byte 0 first, each byte unsigned, MSB first -- the
bit-string order of section "The Other Universal Property"), a proper prefix
before its extensions, and equal strings keep their input order.  Written
with Python's bytes comparison and its stable sort.
"""
from __future__ import annotations

import numpy as np


def strings_of(data: np.ndarray, offsets: np.ndarray) -> list:
    d = bytes(np.asarray(data, dtype=np.uint8))
    o = [int(x) for x in offsets]
    return [d[o[i]:o[i + 1]] for i in range(len(o) - 1)]


def stable_order(data: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """The stable sorting permutation (int64) of the strings."""
    s = strings_of(data, offsets)
    return np.array(sorted(range(len(s)), key=s.__getitem__), dtype=np.int64)


def sort(data: np.ndarray, offsets: np.ndarray, payload: np.ndarray) -> np.ndarray:
    """payload permuted into the strings' sorted order."""
    return np.asarray(payload)[stable_order(data, offsets)]


def pack(strings: list) -> tuple:
    """(data uint8, offsets uint32) of a list of bytes objects."""
    offs = np.zeros(len(strings) + 1, dtype=np.uint32)
    offs[1:] = np.cumsum([len(x) for x in strings])
    return np.frombuffer(b"".join(strings), dtype=np.uint8).copy(), offs
