"""Closed-form grid distances used to pin the oracle.  Test infrastructure.

1. Obstacle-free W x H 4-neighbour grid, every arc weight c:
       d((x1,y1),(x2,y2)) = c * (|x1-x2| + |y1-y2|).
2. Rack layout (blocked columns x % 3 == 2 except on cross rows), every arc
   weight c, both endpoints in aisle columns (x % 3 != 2): if no rack column
   lies strictly between x1 and x2 the Manhattan form holds; otherwise the
   walk must use a cross row r and
       d = c * (|x1-x2| + min_r (|y1-r| + |y2-r|)).
   (Aisle cells of one aisle pair are joined directly; a rack column between
   them can only be crossed on a cross row, and any crossing row costs the
   vertical detour |y1-r| + |y2-r| >= |y1-y2|.)
"""
from __future__ import annotations


def manhattan(x1, y1, x2, y2, c=1):
    return c * (abs(x1 - x2) + abs(y1 - y2))


def rack_distance(x1, y1, x2, y2, cross_rows, c=1):
    lo, hi = min(x1, x2), max(x1, x2)
    blocked_between = any(x % 3 == 2 for x in range(lo + 1, hi))
    if not blocked_between:
        return c * (abs(x1 - x2) + abs(y1 - y2))
    return c * (abs(x1 - x2) + min(abs(y1 - r) + abs(y2 - r) for r in cross_rows))
