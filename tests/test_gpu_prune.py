"""Target-bounded passes (WR_PRUNE_TO_PICKS) on the GPU against the CPU
oracle: orders whose picks lie close together (where the bound prunes most)
and uniform orders, with duplicates, single-pick orders and picks shared by
orders; the pruned matrices equal the oracle's and the pruned solve visits
fewer (tile, block) items.  Misuse is refused."""
import ctypes

import numpy as np
import pytest

import oracle
from wgen import make_config
from wgen.orders import window_orders

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(rt):
    return rt.Context(0)


def _graph(rt, ctx, side):
    wl = make_config("medium", side=side, num_orders=4)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.set_schedule(512, 8, 8)
    G.segment_grid(g.W, g.H, 1, 12, 40)
    return wl, g, G


@pytest.mark.parametrize("capture", [True, False], ids=["replayed", "eager"])
def test_pruned_clustered_orders(rt, ctx, capture):
    wl, g, G = _graph(rt, ctx, 160)
    rng = np.random.default_rng(41)
    off, picks = window_orders(rng, g.aisle_adjacent_vertices(), g.W, g.H, 96, 16, 20)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks)
    full = G.order_matrices(off, picks, algo="overlay", graph_capture=capture)
    v_full = G.last_run()["work_items"]
    got = G.order_matrices(off, picks, algo="overlay", prune=True, graph_capture=capture)
    v_pruned = G.last_run()["work_items"]
    assert (full == exp).all()
    assert (got == exp).all()
    assert v_pruned < 0.7 * v_full, (v_pruned, v_full)
    G.close()


def test_pruned_uniform_orders_with_duplicates(rt, ctx):
    wl, g, G = _graph(rt, ctx, 96)
    rng = np.random.default_rng(42)
    cand = g.aisle_adjacent_vertices()
    sizes = [1, 2, 7, 30, 0, 5, 64]
    orders = [cand[rng.choice(len(cand), P, replace=False)].astype(np.uint32) for P in sizes]
    orders[2][3] = orders[2][1]          # a duplicate pick inside an order
    orders[5][0] = orders[3][4]          # a pick shared by two orders
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    picks = np.concatenate(orders).astype(np.uint32)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks)
    for _ in range(2):   # the second call starts from the first one's replays
        assert (G.order_matrices(off, picks, algo="auto", prune=True) == exp).all()
    G.close()


def test_prune_refuses_misuse(rt, ctx):
    wl, g, G = _graph(rt, ctx, 48)
    off = np.array([0, 3], np.uint32)
    picks = g.aisle_adjacent_vertices()[:3].astype(np.uint32)
    with pytest.raises(rt.WrError) as e:
        G.order_matrices(off, picks, pred=True, algo="overlay", prune=True)
    assert e.value.name == "WR_E_INVALID"
    with pytest.raises(rt.WrError) as e:
        G.order_matrices(off, picks, algo="segmented", prune=True)
    assert e.value.name == "WR_E_UNSUPPORTED"
    d = np.zeros(3 * g.V, np.uint32)
    rc = rt.lib().wr_sssp(G.h, 3, ctypes.c_void_p(picks.ctypes.data), ctypes.c_void_p(d.ctypes.data), None,
                          rt.ALGO["overlay"] | rt.PRUNE_TO_PICKS, None)
    assert rt.STATUS[rc] == "WR_E_INVALID"
    G.close()
