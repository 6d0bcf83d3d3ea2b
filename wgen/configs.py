"""The five synthetic warehouse workloads, as seeded recipes.

Every workload is drawn from ``np.random.default_rng(20655 + index)`` (PCG64)
in a fixed order: edge weights, then workload-specific draws.  Repetition
``rep`` of a workload uses seed ``20655 + index + 1000 * rep``.

  tiny       20x40, cross rows {0,19,39}, w in 1..5, 1 order x 8 picks
  medium     512x512, cross rows every 32 (+ last row), w in 1..10,
             256 orders x 32 picks
  segmented  4096x4096, same layout, w in 1..10, 1024 sources,
             256x256-cell segments
  uneven     2048x2048, w in 1..10, 100k Zipf(1.1) slots, 10k orders with
             Geometric(mean 12) sizes clipped to [2, 64]
  serving    3 levels of 1024x1024, 64 lift sites (w = 50), w in 1..10,
             1% congestion (+0..20) per 100 ms tick, Poisson arrivals,
             sizes uniform in 2..128

``make_config(name, scale=...)`` can shrink the grid side for tests while
keeping the recipe.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .grid import GridGraph, build_grid_graph, cross_rows_every
from .orders import uniform_orders, zipf_orders

BASE_SEED = 20655
CONFIGS = ("tiny", "medium", "segmented", "uneven", "serving")


@dataclass
class Workload:
    name: str
    seed: int
    graph: GridGraph
    pick_offsets: np.ndarray = None   # u32[num_orders+1]
    picks: np.ndarray = None          # u32[sum P]
    sources: np.ndarray = None        # u32[S] (segmented workload)
    segment_tile: tuple = None        # (tile_w, tile_h)
    slots: np.ndarray = None
    extra: dict = field(default_factory=dict)

    @property
    def num_orders(self) -> int:
        return 0 if self.pick_offsets is None else len(self.pick_offsets) - 1


def make_config(name: str, rep: int = 0, side: int | None = None,
                num_orders: int | None = None, num_sources: int | None = None) -> Workload:
    idx = CONFIGS.index(name)
    seed = BASE_SEED + idx + 1000 * rep
    rng = np.random.default_rng(seed)
    if name == "tiny":
        g = build_grid_graph(20, 40, [0, 19, 39], 1, 5, rng)
        off, picks = uniform_orders(rng, g.aisle_adjacent_vertices(),
                                    num_orders or 1, 8)
        return Workload(name, seed, g, off, picks)
    if name == "medium":
        n = side or 512
        g = build_grid_graph(n, n, cross_rows_every(n, 32), 1, 10, rng)
        off, picks = uniform_orders(rng, g.aisle_adjacent_vertices(),
                                    num_orders or 256, 32)
        return Workload(name, seed, g, off, picks)
    if name == "segmented":
        n = side or 4096
        g = build_grid_graph(n, n, cross_rows_every(n, 32), 1, 10, rng)
        cand = g.aisle_adjacent_vertices()
        S = num_sources or 1024
        src = cand[rng.choice(len(cand), size=S, replace=False)].astype(np.uint32)
        tile = 256 if n >= 1024 else max(16, n // 16)
        return Workload(name, seed, g, sources=src, segment_tile=(tile, tile))
    if name == "uneven":
        n = side or 2048
        g = build_grid_graph(n, n, cross_rows_every(n, 32), 1, 10, rng)
        cand = g.aisle_adjacent_vertices()
        n_slots = min(100_000, len(cand))
        off, picks, slots = zipf_orders(rng, cand, n_slots, 1.1,
                                        num_orders or 10_000, 12.0, 2, 64)
        return Workload(name, seed, g, off, picks, slots=slots)
    if name == "serving":
        n = side or 1024
        levels = 3
        # lift sites are drawn before the weights so that the layout is fixed
        from .grid import rack_layout
        blocked = rack_layout(n, n, cross_rows_every(n, 32))
        free = np.flatnonzero(~blocked.ravel())
        site = free[rng.choice(len(free), size=min(64, len(free)), replace=False)]
        sy, sx = np.divmod(site, n)
        g = build_grid_graph(n, n, cross_rows_every(n, 32), 1, 10, rng,
                             levels=levels, lift_sites=(sx, sy), lift_w=50)
        return Workload(name, seed, g, extra={"lift_sites": (sx, sy),
                                              "pick_lo": 2, "pick_hi": 128,
                                              "rates": (500, 2000, 8000),
                                              "tick_s": 0.1, "congestion": 0.01,
                                              "congestion_extra": 20})
    raise ValueError(name)
