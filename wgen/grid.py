"""Warehouse grid graphs in CSR form.

A warehouse level is a W x H grid of cells (x = column, y = row, vertex id
``level*W*H + y*W + x``).  Racks are blocked cells in every third column
(``x % 3 == 2``) except on cross-aisle rows, which leaves two-wide aisles.
Free cells are joined to their free 4-neighbours by two directed arcs that
carry the same weight (one draw per undirected edge).  Blocked cells keep
their vertex ids but have no arcs.  Levels of a multi-level warehouse are
joined by lift arcs at fixed (x, y) sites.

The paper models the floor as integer (i, j) stop coordinates over racks
(state space and routes-and-clusters subsections of the mathematical model)
and routes between stops over a directed weighted graph held as integer
arrays (GPU implementation subsection); the rack/aisle geometry below is the
synthetic stand-in for the paper's unpublished instance graphs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Direction order inside one CSR row: targets sorted by ascending vertex id.
#   lift-down (-W*H), up (-W), left (-1), right (+1), down (+W), lift-up (+W*H)


def cross_rows_every(H: int, every: int, include_last: bool = True) -> list[int]:
    """Cross-aisle rows {y : y % every == 0}, plus the last row H-1."""
    rows = set(range(0, H, every))
    if include_last:
        rows.add(H - 1)
    return sorted(rows)


def rack_layout(W: int, H: int, cross_rows) -> np.ndarray:
    """Boolean [H, W] array, True where the cell is a blocked rack cell."""
    blocked = np.zeros((H, W), dtype=bool)
    blocked[:, (np.arange(W) % 3) == 2] = True
    rows = np.asarray(list(cross_rows), dtype=np.int64)
    if rows.size:
        blocked[rows, :] = False
    return blocked


def free_mask(blocked: np.ndarray) -> np.ndarray:
    return ~blocked


def aisle_adjacent_mask(blocked: np.ndarray) -> np.ndarray:
    """Free cells with at least one blocked 4-neighbour (grid edge excluded)."""
    nb = np.zeros_like(blocked)
    nb[:, 1:] |= blocked[:, :-1]
    nb[:, :-1] |= blocked[:, 1:]
    nb[1:, :] |= blocked[:-1, :]
    nb[:-1, :] |= blocked[1:, :]
    return (~blocked) & nb


@dataclass
class GridGraph:
    """A warehouse graph in CSR form plus the geometry that produced it."""

    W: int
    H: int
    levels: int
    blocked: np.ndarray            # [H, W] bool (same on every level)
    row_ptr: np.ndarray            # uint32[V+1]
    col: np.ndarray                # uint32[E]
    w: np.ndarray                  # uint32[E]
    # undirected edges: CSR positions of the two arcs and the drawn base weight
    edge_arc_a: np.ndarray = field(repr=False, default=None)
    edge_arc_b: np.ndarray = field(repr=False, default=None)
    edge_base_w: np.ndarray = field(repr=False, default=None)
    edge_is_lift: np.ndarray = field(repr=False, default=None)

    @property
    def V(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def E(self) -> int:
        return int(self.col.shape[0])

    def vid(self, x, y, level=0):
        return level * self.W * self.H + np.asarray(y) * self.W + np.asarray(x)

    def xy(self, v):
        v = np.asarray(v, dtype=np.int64)
        plane = self.W * self.H
        level, r = np.divmod(v, plane)
        y, x = np.divmod(r, self.W)
        return x, y, level

    def free_vertices(self) -> np.ndarray:
        f = np.flatnonzero(~self.blocked.ravel())
        plane = self.W * self.H
        return np.concatenate([f + l * plane for l in range(self.levels)]).astype(np.int64)

    def aisle_adjacent_vertices(self) -> np.ndarray:
        a = np.flatnonzero(aisle_adjacent_mask(self.blocked).ravel())
        plane = self.W * self.H
        return np.concatenate([a + l * plane for l in range(self.levels)]).astype(np.int64)


def build_grid_graph(W: int, H: int, cross_rows, wmin: int, wmax: int,
                     rng: np.random.Generator, levels: int = 1,
                     lift_sites=None, lift_w: int = 50) -> GridGraph:
    """Build the CSR of a (multi-level) rack warehouse.

    Weights: one uniform integer draw in [wmin, wmax] for every potential
    horizontal edge of every level (array [levels, H, W-1]), then every
    potential vertical edge ([levels, H-1, W]), in that order, whether or not
    both cells are free; an edge exists when both of its cells are free.
    Lift edges get the fixed weight ``lift_w``.
    """
    blocked = rack_layout(W, H, cross_rows)
    free = ~blocked
    plane = W * H
    V = plane * levels
    wh = rng.integers(wmin, wmax + 1, size=(levels, H, W - 1), dtype=np.int64)
    wv = rng.integers(wmin, wmax + 1, size=(levels, H - 1, W), dtype=np.int64)

    h_ok = free[:, :-1] & free[:, 1:]          # edge (x,y)-(x+1,y)
    v_ok = free[:-1, :] & free[1:, :]          # edge (x,y)-(x,y+1)

    lift = np.zeros((H, W), dtype=bool)
    if lift_sites is not None and levels > 1:
        lx, ly = lift_sites
        lift[ly, lx] = True
        assert not blocked[ly, lx].any(), "lift sites must be free cells"

    # per-cell flags for each direction, per level (identical across levels
    # except the lift directions at the bottom / top level)
    has_up = np.zeros((H, W), dtype=bool)
    has_up[1:, :] = v_ok
    has_down = np.zeros((H, W), dtype=bool)
    has_down[:-1, :] = v_ok
    has_left = np.zeros((H, W), dtype=bool)
    has_left[:, 1:] = h_ok
    has_right = np.zeros((H, W), dtype=bool)
    has_right[:, :-1] = h_ok

    dirs = []  # (flag[levels,H,W], delta, weight[levels,H,W])
    L = levels
    z = np.zeros((L, H, W), dtype=np.int64)
    # weight of each directed arc leaving cell (x,y)
    w_up = z.copy(); w_up[:, 1:, :] = wv
    w_down = z.copy(); w_down[:, :-1, :] = wv
    w_left = z.copy(); w_left[:, :, 1:] = wh
    w_right = z.copy(); w_right[:, :, :-1] = wh
    lift_dn = np.zeros((L, H, W), dtype=bool)
    lift_upf = np.zeros((L, H, W), dtype=bool)
    if L > 1:
        lift_dn[1:] = lift[None]
        lift_upf[:-1] = lift[None]
    wl = np.full((L, H, W), lift_w, dtype=np.int64)
    dirs.append((lift_dn, -plane, wl))
    dirs.append((np.broadcast_to(has_up, (L, H, W)), -W, w_up))
    dirs.append((np.broadcast_to(has_left, (L, H, W)), -1, w_left))
    dirs.append((np.broadcast_to(has_right, (L, H, W)), +1, w_right))
    dirs.append((np.broadcast_to(has_down, (L, H, W)), +W, w_down))
    dirs.append((lift_upf, +plane, wl))

    deg = np.zeros(V, dtype=np.int64)
    for f, _, _ in dirs:
        deg += f.reshape(-1)
    row_ptr = np.zeros(V + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    E = int(row_ptr[-1])
    col = np.empty(E, dtype=np.uint32)
    w = np.empty(E, dtype=np.uint32)
    fill = row_ptr[:-1].copy()
    ids = np.arange(V, dtype=np.int64)
    arc_pos = {}
    for k, (f, delta, wt) in enumerate(dirs):
        fl = f.reshape(-1)
        src = ids[fl]
        pos = fill[fl]
        col[pos] = (src + delta).astype(np.uint32)
        w[pos] = wt.reshape(-1)[fl].astype(np.uint32)
        fill[fl] += 1
        arc_pos[k] = (src, pos)

    # undirected edges: pair each "right"/"down"/"lift-up" arc with its reverse
    def _pair(k_fwd, k_bwd, delta, is_lift):
        src_f, pos_f = arc_pos[k_fwd]
        src_b, pos_b = arc_pos[k_bwd]
        lookup = np.full(V, -1, dtype=np.int64)
        lookup[src_b] = pos_b
        rev = lookup[src_f + delta]
        assert (rev >= 0).all()
        return pos_f, rev, w[pos_f].astype(np.int64), np.full(len(pos_f), is_lift)

    parts = [_pair(3, 2, +1, False), _pair(4, 1, +W, False)]
    if L > 1:
        parts.append(_pair(5, 0, +plane, True))
    ea = np.concatenate([p[0] for p in parts])
    eb = np.concatenate([p[1] for p in parts])
    ew = np.concatenate([p[2] for p in parts])
    el = np.concatenate([p[3] for p in parts])
    return GridGraph(W=W, H=H, levels=levels, blocked=blocked,
                     row_ptr=row_ptr.astype(np.uint32), col=col, w=w,
                     edge_arc_a=ea, edge_arc_b=eb, edge_base_w=ew,
                     edge_is_lift=el)
