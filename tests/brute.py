"""Brute force for tiny alignments: enumerate every local alignment path.

Independent of any dynamic programming: each path is a start on an aligned pair
followed by a sequence of moves (pair, query-gap, database-gap); its score is
summed move by move, a run of gap moves in one direction costing
open + length * extend.  Paths may be confined to a band of cells.
"""
from __future__ import annotations


def enumerate_local(q: str, s: str, match: int, mismatch: int, gap_open: int, gap_extend: int,
                    in_band=None):
    """Return (best score, set of optimal spans (q_start, q_end, d_start, d_end)).

    A span ends on an aligned pair.  ``in_band(i, j)`` restricts every visited cell,
    where cell (i, j) means query base i and database base j were the last consumed.
    The empty alignment scores 0 with no span.
    """
    R, C = len(q), len(s)
    best = 0
    spans = set()
    ok = in_band or (lambda i, j: True)

    def sigma(i, j):
        return match if q[i] == s[j] else -mismatch

    def walk(i0, j0, i, j, score, last):
        nonlocal best, spans
        if last == "M":
            if score > best:
                best = score
                spans = {(i0, i + 1, j0, j + 1)}
            elif score == best and score > 0:
                spans.add((i0, i + 1, j0, j + 1))
        # pair
        if i + 1 < R and j + 1 < C and ok(i + 1, j + 1):
            walk(i0, j0, i + 1, j + 1, score + sigma(i + 1, j + 1), "M")
        # database base against a gap (moves right)
        if j + 1 < C and ok(i, j + 1):
            cost = gap_extend if last == "D" else gap_open + gap_extend
            walk(i0, j0, i, j + 1, score - cost, "D")
        # query base against a gap (moves down)
        if i + 1 < R and ok(i + 1, j):
            cost = gap_extend if last == "I" else gap_open + gap_extend
            walk(i0, j0, i + 1, j, score - cost, "I")

    for i0 in range(R):
        for j0 in range(C):
            if ok(i0, j0):
                walk(i0, j0, i0, j0, sigma(i0, j0), "M")
    return best, spans
