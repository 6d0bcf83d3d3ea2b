"""Seeded order streams: pick lists, popularity-driven orders, arrivals and
congestion ticks.

An order is a list of pick vertices (the stops of one route; the paper's
routes-and-clusters subsection collapses the picking nodes of one rack onto
its stop, so a pick here is a stop vertex).  Picks are drawn without
replacement within one order.
"""
from __future__ import annotations

import numpy as np


def _offsets(sizes) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.uint32)
    off[1:] = np.cumsum(np.asarray(sizes, dtype=np.int64)).astype(np.uint32)
    return off


def uniform_orders(rng: np.random.Generator, candidates: np.ndarray,
                   num_orders: int, sizes) -> tuple[np.ndarray, np.ndarray]:
    """``num_orders`` orders; order k has ``sizes[k]`` distinct picks drawn
    uniformly from ``candidates``.  Returns (pick_offsets u32[n+1], picks u32).
    """
    sizes = np.broadcast_to(np.asarray(sizes, dtype=np.int64), (num_orders,))
    picks = []
    for k in range(num_orders):
        idx = rng.choice(len(candidates), size=int(sizes[k]), replace=False)
        picks.append(candidates[idx])
    flat = (np.concatenate(picks) if picks else np.zeros(0)).astype(np.uint32)
    return _offsets(sizes), flat


def window_orders(rng: np.random.Generator, candidates: np.ndarray, W: int, H: int,
                  num_orders: int, size: int, window: int) -> tuple[np.ndarray, np.ndarray]:
    """Orders whose picks lie close together, as after the paper's clustering
    reorganisation has gathered an order's articles: order k takes ``size``
    distinct picks uniformly from the candidates inside a ``window`` x
    ``window`` cell square placed uniformly on the W x H grid (the square
    grows until it holds enough candidates).  Returns (pick_offsets, picks).
    """
    cx, cy = candidates % W, candidates // W
    picks = []
    for _ in range(num_orders):
        x0 = int(rng.integers(0, max(1, W - window + 1)))
        y0 = int(rng.integers(0, max(1, H - window + 1)))
        r = window
        while True:
            inside = np.flatnonzero((cx >= x0) & (cx < x0 + r) & (cy >= y0) & (cy < y0 + r))
            if len(inside) >= size or r >= max(W, H):
                break
            r *= 2
        idx = rng.choice(inside, size=min(size, len(inside)), replace=False)
        picks.append(candidates[idx])
    sizes = [len(p) for p in picks]
    flat = (np.concatenate(picks) if picks else np.zeros(0)).astype(np.uint32)
    return _offsets(sizes), flat


def zipf_popularity(n_ranks: int, s: float) -> np.ndarray:
    """Finite Zipf law over ranks 1..n: p_k proportional to k^-s."""
    p = np.arange(1, n_ranks + 1, dtype=np.float64) ** (-s)
    return p / p.sum()


def geometric_clipped(rng, mean: float, lo: int, hi: int, n: int) -> np.ndarray:
    """Geometric on {1,2,...} with success probability 1/mean, clipped."""
    g = rng.geometric(1.0 / mean, size=n)
    return np.clip(g, lo, hi).astype(np.int64)


def zipf_orders(rng: np.random.Generator, candidates: np.ndarray, n_slots: int,
                s: float, num_orders: int, mean_size: float, lo: int, hi: int):
    """Popularity-driven orders.

    ``n_slots`` distinct slot cells are drawn uniformly from ``candidates``;
    product rank k (1 = most popular) is placed at slot ``perm[k-1]`` for a
    seeded random permutation; pick-list sizes are Geometric(1/mean) clipped
    to [lo, hi]; each order draws its picks by popularity, without
    replacement within the order (duplicate draws are rejected).
    Returns (pick_offsets, picks, slots).
    """
    slots = candidates[rng.choice(len(candidates), size=n_slots, replace=False)]
    perm = rng.permutation(n_slots)
    cdf = np.cumsum(zipf_popularity(n_slots, s))
    cdf[-1] = 1.0
    sizes = geometric_clipped(rng, mean_size, lo, hi, num_orders)
    picks = []
    for k in range(num_orders):
        P = int(sizes[k])
        got: list[int] = []
        seen: set[int] = set()
        while len(got) < P:
            r = np.searchsorted(cdf, rng.random(2 * P), side="right")
            for rank in r.tolist():
                if rank not in seen:
                    seen.add(rank)
                    got.append(rank)
                    if len(got) == P:
                        break
        picks.append(slots[perm[np.asarray(got)]])
    flat = np.concatenate(picks).astype(np.uint32)
    return _offsets(sizes), flat, slots


def poisson_arrivals(rng: np.random.Generator, rate_per_s: float, n: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


class CongestionTicker:
    """Time-varying aisle weights.

    Every tick picks a fraction of the undirected non-lift edges uniformly
    and sets both of their arcs to base + U{0..extra_max}; the edges picked at
    the previous tick revert to their base weight (the change is not
    cumulative).  ``tick()`` returns (arc_index u32, new_w u32) covering the
    reverts followed by the new picks (a later entry for the same arc wins).
    """

    def __init__(self, rng, edge_arc_a, edge_arc_b, edge_base_w, edge_is_lift,
                 fraction: float = 0.01, extra_max: int = 20):
        self.rng = rng
        keep = ~np.asarray(edge_is_lift, dtype=bool)
        self.a = np.asarray(edge_arc_a)[keep]
        self.b = np.asarray(edge_arc_b)[keep]
        self.base = np.asarray(edge_base_w)[keep]
        self.k = max(1, int(round(fraction * len(self.a))))
        self.extra_max = extra_max
        self.prev = np.zeros(0, dtype=np.int64)

    def tick(self):
        rev = self.prev
        pick = self.rng.choice(len(self.a), size=self.k, replace=False)
        neww = self.base[pick] + self.rng.integers(0, self.extra_max + 1, size=self.k)
        arcs = np.concatenate([self.a[rev], self.b[rev], self.a[pick], self.b[pick]])
        vals = np.concatenate([self.base[rev], self.base[rev], neww, neww])
        self.prev = pick
        return arcs.astype(np.uint32), vals.astype(np.uint32)
