"""Brute-force shortest distances by enumerating every simple path.

Test infrastructure only.  For a tiny directed graph (V <= 9) the minimum over
all simple s->v paths of the summed arc weights is the definition of d(s, v)
for non-negative weights (a shortest walk can always drop its cycles).  Pure
Python, exponential, independent of the C oracle.
"""
from __future__ import annotations

INF = 0xFFFFFFFF


def all_pairs_by_enumeration(V: int, arcs) -> list[list[int]]:
    """arcs: iterable of (u, v, w).  Returns D[s][v] (INF if unreachable)."""
    out_arcs = [[] for _ in range(V)]
    for u, v, w in arcs:
        out_arcs[u].append((v, w))
    D = [[INF] * V for _ in range(V)]
    for s in range(V):
        best = D[s]
        best[s] = 0
        on_path = [False] * V

        def walk(u, length):
            on_path[u] = True
            if length < best[u]:
                best[u] = length
            for v, w in out_arcs[u]:
                if not on_path[v]:
                    walk(v, length + w)
            on_path[u] = False

        walk(s, 0)
    return D


def route_by_enumeration(D) -> tuple[int, list[int]]:
    """Optimal open route over the stops of a tiny n x n matrix by trying
    every ordering (n <= 8): the length is the sum of the n-1 steps along the
    ordering (infinite if a step is INF), and among the shortest orderings
    the lexicographically smallest is kept -- permutations() yields them in
    lexicographic order, so the first strict improvement wins.  Returns
    (length or None when every ordering is infinite, ordering)."""
    import itertools
    n = len(D)
    best, best_p = None, list(range(n))
    for p in itertools.permutations(range(n)):
        length = 0
        for a, b in zip(p, p[1:]):
            if D[a][b] == INF:
                length = None
                break
            length += D[a][b]
        if length is not None and (best is None or length < best):
            best, best_p = length, list(p)
    return best, best_p
