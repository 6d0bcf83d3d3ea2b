"""Failure handling on the GPU, forced from the host: wr_debug_fault makes
the library's next device allocation or kernel launch fail before anything
reaches the device (no kernel faults).  A failed call reports its status and
the next call on the same graph is exact; a server step that fails fails the
orders it held and serving goes on with exact results."""
import numpy as np
import pytest

import oracle
from wgen import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(rt):
    return rt.Context(0)


@pytest.fixture(autouse=True)
def disarm(rt):
    yield
    rt.debug_fault("off")


def _graph(rt, ctx, side=64, orders=6):
    wl = make_config("medium", side=side, num_orders=orders)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 12, 20)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    return wl, G, exp


@pytest.mark.parametrize("capture", [True, False], ids=["replayed", "eager"])
@pytest.mark.parametrize("nth", [1, 3, 6])
def test_launch_failure_then_exact(rt, ctx, capture, nth):
    """A launch failing at the nth launch of a call (a fill, a seed or, with
    eager passes, a pass in the middle of the solve) fails that call with
    WR_E_DEVICE; the next call is exact."""
    wl, G, exp = _graph(rt, ctx)
    off, picks = wl.pick_offsets, wl.picks
    assert (G.order_matrices(off, picks, algo="overlay", graph_capture=capture) == exp).all()
    rt.debug_fault("launch", nth)
    with pytest.raises(rt.WrError) as e:
        G.order_matrices(off, picks, algo="overlay", graph_capture=capture)
    assert e.value.name == "WR_E_DEVICE"
    for _ in range(2):
        assert (G.order_matrices(off, picks, algo="overlay", graph_capture=capture) == exp).all()
    G.close()


def test_allocation_failure_then_exact(rt, ctx):
    """An allocation failing while a graph is created, and while a call sizes
    its work buffers, fails those calls with WR_E_NOMEM; retries succeed."""
    wl = make_config("medium", side=64, num_orders=6)
    g = wl.graph
    rt.debug_fault("alloc", 2)
    with pytest.raises(rt.WrError) as e:
        rt.Graph(ctx, g.row_ptr, g.col, g.w)
    assert e.value.name == "WR_E_NOMEM"
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 12, 20)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    rt.debug_fault("alloc", 1)
    with pytest.raises(rt.WrError) as e:
        G.order_matrices(wl.pick_offsets, wl.picks, algo="overlay")
    assert e.value.name == "WR_E_NOMEM"
    assert (G.order_matrices(wl.pick_offsets, wl.picks, algo="overlay") == exp).all()
    G.close()


def _expect(g, picks):
    P = len(picks)
    return oracle.order_matrices(g.row_ptr, g.col, g.w, np.array([0, P], np.uint32), picks).reshape(P, P)


@pytest.mark.parametrize("nth", [1, 2, 5])
def test_server_step_failure_fails_its_orders_only(rt, ctx, nth):
    """An allocation failing inside a scheduler step (admission or read-out)
    fails the orders that step held, with WR_E_NOMEM; orders submitted
    afterwards are served exactly, and so are the ones served before."""
    wl = make_config("medium", side=64, num_orders=15)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 12, 20)
    off = wl.pick_offsets
    orders = [wl.picks[off[o]:off[o + 1]].copy() for o in range(len(off) - 1)]
    srv = rt.Server(G)
    first = [srv.submit(o) for o in orders[:5]]
    srv.drain()
    for t, o in zip(first, orders[:5]):
        D, info = srv.poll(t)
        assert info["status"] == 0 and (D == _expect(g, o)).all()
    rt.debug_fault("alloc", nth)
    hit = [srv.submit(o) for o in orders[5:10]]
    srv.drain()
    failed = 0
    for t, o in zip(hit, orders[5:10]):
        try:
            D, info = srv.poll(t)
            assert (D == _expect(g, o)).all()
        except rt.WrError as e:
            assert e.name == "WR_E_NOMEM"
            failed += 1
    assert failed >= 1
    rt.debug_fault("off")
    later = [srv.submit(o) for o in orders[10:]]
    srv.drain()
    for t, o in zip(later, orders[10:]):
        D, info = srv.poll(t)
        assert info["status"] == 0 and (D == _expect(g, o)).all()
    assert srv.stats()["failed"] == failed
    srv.close()
    G.close()
