"""The paper's own in-place exchange partition -- TEST INFRASTRUCTURE ONLY.

Written from the prose of section "Operation of Algorithm": the element at
the lower position is the working element; its bit (section "Bit
Extraction", bit 0 = most significant) either leaves it in the lower
sub-array (lower bound moves up) or exchanges it with the element at the
upper bound (upper bound moves down), until the bounds cross (section
"Partition Repetition").  If every element stayed low the call continues on
the same bounds with the next bit ("pass-through"); otherwise it continues on
both sub-arrays (section "Determine Recursive Call on Sub-arrays").  The
recursion stops at one element or when the bits are used up (section
"Evaluate for Recursive Base Case").

The exchange makes this partition unstable (section "Conclusion"); it serves
only to check the paper's printed configurations and that its key order
agrees with the stable oracle.
"""
from __future__ import annotations


def _bit(value: int, width: int, b: int) -> int:
    return (value >> (width - 1 - b)) & 1


def binar_swap_sort(values: list[int], width: int, trace=None, payload=None) -> list[int]:
    """Sort a list of ``width``-bit unsigned integers in place, unstably.

    ``payload`` (optional list) is exchanged along with the values.

    ``trace`` (optional list) receives, for each partition call, a record
    ``(bit, lower, upper, states)`` where ``states`` lists the configuration
    (lower sub-array, unplaced, upper sub-array) before the first placement
    and after each placement.
    """
    a = values

    def rec(lower: int, upper: int, b: int) -> None:  # inclusive bounds
        if b >= width or upper < lower + 1:
            return
        lo, hi = lower, upper
        states = [(a[lower:lo], a[lo:hi + 1], a[hi + 1:upper + 1])]
        while lo <= hi:
            if _bit(a[lo], width, b) == 0:
                lo += 1
            else:
                a[lo], a[hi] = a[hi], a[lo]
                if payload is not None:
                    payload[lo], payload[hi] = payload[hi], payload[lo]
                hi -= 1
            states.append((a[lower:lo], a[lo:hi + 1], a[hi + 1:upper + 1]))
        if trace is not None:
            trace.append((b, lower, upper, [tuple(list(s) for s in st) for st in states]))
        if lo == upper + 1:
            rec(lower, upper, b + 1)
        else:
            rec(lower, lo - 1, b + 1)
            rec(lo, upper, b + 1)

    rec(0, len(a) - 1, 0)
    return a
