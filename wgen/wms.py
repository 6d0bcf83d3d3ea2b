"""Seeded inputs of the warehouse reorganisation loop (the WMS/RDS model):
initial warehouse states and per-iteration picking orders.  Inputs only;
the loop itself is computed elsewhere.

A warehouse has nx x ny x nz nodes (rack (i, j), shelf k), node id
v = (k * ny + j) * nx + i.  An initial state leaves `empty_racks` racks
(every shelf of them) empty and gives each other node its own article type
(1..N, a random permutation), fully stocked at `mmax` parcels.  A picking
order is `po` purchase orders (20 in the paper's experiments) of `per_po`
distinct article types each (10; all po * per_po types drawn without
replacement), with 1..mmax parcels of each.  Per iteration the order is
either the same (experiment 1), or has the first article of each purchase
order replaced by a uniform random type (experiment 2), or a uniformly
chosen article of each purchase order replaced (experiment 3).  The parcels
are fixed per run, or drawn afresh per iteration with `qty_per_iter`.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PURCHASE_ORDERS = 20
ARTICLES_PER_PO = 10


@dataclass
class WmsSetup:
    nx: int
    ny: int
    nz: int
    mmax: int
    n_articles: int
    A0: np.ndarray       # u32[runs, V] article per node (0 = empty)
    M0: np.ndarray       # u32[runs, V] balance per node
    orders: np.ndarray   # u32[runs, iters, po * per_po] article per (purchase order, slot)
    qty: np.ndarray      # u32[runs, po * per_po] parcels per slot, or u32[runs, iters, po * per_po]
    po: int = PURCHASE_ORDERS
    k: int = 3           # clusters

    @property
    def V(self) -> int:
        return self.nx * self.ny * self.nz


def make_wms(seed: int, nx: int, ny: int, nz: int, empty_racks: int, runs: int, iters: int,
             experiment: int, mmax: int = 10, po: int = PURCHASE_ORDERS, per_po: int = ARTICLES_PER_PO,
             k: int = 3, qty_per_iter: bool = False) -> WmsSetup:
    rng = np.random.default_rng(seed)
    V = nx * ny * nz
    N = V - empty_racks * nz
    P = po * per_po
    A0 = np.zeros((runs, V), np.uint32)
    M0 = np.zeros((runs, V), np.uint32)
    orders = np.zeros((runs, iters, P), np.uint32)
    qty = np.zeros((runs, iters, P) if qty_per_iter else (runs, P), np.uint32)
    for r in range(runs):
        racks = rng.choice(nx * ny, size=empty_racks, replace=False)
        empty = np.zeros(nx * ny, bool)
        empty[racks] = True
        full = ~np.tile(empty, nz)     # node v = k * (nx * ny) + rack
        A0[r][full] = rng.permutation(N) + 1
        M0[r][full] = mmax
        base = rng.choice(N, size=P, replace=False) + 1
        qty[r] = rng.integers(1, mmax + 1, size=qty[r].shape)
        o = np.broadcast_to(base.reshape(1, po, per_po), (iters, po, per_po)).copy()
        if experiment == 2:
            o[:, :, 0] = rng.integers(1, N + 1, size=(iters, po))
        elif experiment == 3:
            slot = rng.integers(0, per_po, size=(iters, po))
            o[np.arange(iters)[:, None], np.arange(po)[None, :], slot] = rng.integers(1, N + 1, size=(iters, po))
        orders[r] = o.reshape(iters, P)
    return WmsSetup(nx, ny, nz, mmax, N, A0, M0, orders, qty, po, k)
