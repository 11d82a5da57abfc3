"""The paper's own in-place exchange partition -- TEST INFRASTRUCTURE ONLY.

Restated from the prose of section "Operation of Algorithm" and section
"Partition Repetition": a sub-array is split on one bit (section "Bit
Extraction", bit 0 = most significant) by moving a front cursor up over
elements whose bit is 0, and sending each element whose bit is 1 to the back,
where it changes places with the element that stood there; the back boundary
then moves down and the element that arrived is examined next.  When the two
cursors meet, the front part holds the 0s and the back part the 1s.  If one
part is empty the same bounds continue with the next bit (pass-through,
section "Optimize the Algorithm"); otherwise both parts continue with the
next bit (section "Determine Recursive Call on Sub-arrays").  A part of one
element, or a bit index past the key width, is finished (section "Evaluate
for Recursive Base Case").

Here the recursion is an explicit work stack of half-open ranges.  The
exchange makes the partition unstable (section "Conclusion"); this module
serves only to check the paper's printed configurations and that its key
order agrees with the stable oracle.
"""
from __future__ import annotations


def binar_swap_sort(values: list[int], width: int, trace=None, payload=None) -> list[int]:
    """Sort a list of ``width``-bit unsigned integers in place, unstably.

    ``payload`` (optional list) changes places along with the values.

    ``trace`` (optional list) receives one record per split,
    ``(bit, first, last, states)`` with inclusive bounds ``first..last`` as
    the paper prints them, where ``states`` lists the configuration (0s
    placed, not yet examined, 1s placed) before the first step and after
    every step.
    """
    a = values
    shift = [width - 1 - b for b in range(width)]

    def exchange(i: int, j: int) -> None:
        a[i], a[j] = a[j], a[i]
        if payload is not None:
            payload[i], payload[j] = payload[j], payload[i]

    work = [(0, len(a), 0)]                # (start, stop exclusive, bit)
    while work:
        start, stop, bit = work.pop()
        if stop - start < 2 or bit >= width:
            continue
        front, back = start, stop           # [start, front) holds 0s, [back, stop) holds 1s
        snap = lambda: (a[start:front], a[front:back], a[back:stop])  # noqa: E731
        states = [snap()]
        while front != back:
            if (a[front] >> shift[bit]) & 1:
                back -= 1
                exchange(front, back)
            else:
                front += 1
            states.append(snap())
        if trace is not None:
            trace.append((bit, start, stop - 1, [tuple(list(part) for part in st) for st in states]))
        if front in (start, stop):
            work.append((start, stop, bit + 1))       # one side empty: same bounds, next bit
        else:
            work.append((front, stop, bit + 1))       # the 1s, taken after
            work.append((start, front, bit + 1))      # the 0s, taken first
    return a
