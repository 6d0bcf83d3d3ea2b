"""Seeded random graph builders for tests (inputs only, no routing math)."""
import numpy as np


def random_csr(rng, V, E, wmax=9, zero_frac=0.0, self_loops=True):
    u = rng.integers(0, V, size=E)
    v = rng.integers(0, V, size=E)
    if not self_loops:
        keep = u != v
        u, v = u[keep], v[keep]
    w = rng.integers(1, wmax + 1, size=len(u))
    if zero_frac > 0:
        w[rng.random(len(u)) < zero_frac] = 0
    order = np.lexsort((v, u))
    u, v, w = u[order], v[order], w[order]
    row_ptr = np.zeros(V + 1, dtype=np.uint32)
    np.add.at(row_ptr, u + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.uint32)
    return row_ptr, v.astype(np.uint32), w.astype(np.uint32)


def csr_arcs(row_ptr, col, w):
    V = len(row_ptr) - 1
    for u in range(V):
        for e in range(int(row_ptr[u]), int(row_ptr[u + 1])):
            yield u, int(col[e]), int(w[e])
