"""The library's unchanged HIP kernels and host runtime, run on the CPU by the
test executor (tests/simt_cpu: lanes as threads, emulated wave collectives
and barriers, AddressSanitizer on every buffer), against the oracle.  This
checks the kernels' logic and bounds without a GPU; the GPU tests check the
same paths on the hardware."""
import numpy as np
import pytest

import oracle
from wgen import make_config

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def harness():
    from tests.simt_cpu import harness as h
    h.driver(rebuild=True)
    return h


def test_overlay_order_matrices_tiny(harness):
    wl = make_config("tiny")
    g = wl.graph
    st, out, _, err = harness.run(g.row_ptr, g.col, g.w, pick_offsets=wl.pick_offsets, picks=wl.picks,
                                  algo="overlay", seg=("grid", g.W, g.H, 1, g.W // 3, g.H // 3))
    assert st == 0, err[-2000:]
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (out == exp).all()


def test_segmented_rows_and_pred_random_graph(harness):
    from tests.helpers import random_csr
    rng = np.random.default_rng(31)
    V = 160
    rp, col, w = random_csr(rng, V, 4 * V, wmax=20)
    seg = rng.integers(0, 5, V).astype(np.uint32)
    src = rng.choice(V, 9, replace=False).astype(np.uint32)
    st, out, pred, err = harness.run(rp, col, w, sources=src, algo="segmented", pred=True,
                                     seg=("map", 5, seg))
    assert st == 0, err[-2000:]
    d = out.reshape(len(src), V)
    p = pred.reshape(len(src), V)
    for i, s in enumerate(src):
        ed = oracle.dijkstra(rp, col, w, int(s))
        assert (d[i] == ed).all()
        assert (p[i] == oracle.canonical_pred(rp, col, w, int(s), ed)).all()


def test_order_routes_over_executor_matrices(harness):
    """wr_order_routes (subset programme in LDS) over the library's own
    matrices for orders of 0..12 stops with duplicate picks: lengths and
    orderings equal the oracle's, with every LDS and global access checked."""
    wl = make_config("medium", side=24, num_orders=8)
    g = wl.graph
    rng = np.random.default_rng(3)
    sizes = [0, 1, 2, 3, 5, 8, 12, 7, 12, 4]
    picks = np.concatenate([rng.choice(wl.picks, s) for s in sizes]).astype(np.uint32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    st, out, _, err = harness.run(g.row_ptr, g.col, g.w, pick_offsets=off, picks=picks, algo="overlay",
                                  seg=("grid", g.W, g.H, 1, 8, 8), routes=True)
    assert st == 0, err[-2000:]
    ncell = int((np.diff(off.astype(np.int64)) ** 2).sum())
    mats = out[:ncell]
    words = out[ncell:ncell + 2 * len(sizes)].astype(np.uint64)
    lens = words[0::2] | (words[1::2] << np.uint64(32))
    rts = out[ncell + 2 * len(sizes):]
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks)
    assert (mats == exp).all()
    el, er = oracle.order_routes(off, exp)
    assert (lens == el).all() and (rts == er).all()


def test_clustered_routes_over_executor_matrices(harness):
    """wr_order_routes_clustered (K-means in wave 0, the per-cluster and the
    chaining subset programmes) over executor-computed matrices, orders of
    0..32 picks at m = 10 (the largest chaining programme): lengths,
    orderings and cluster counts equal the oracle's."""
    wl = make_config("medium", side=24, num_orders=8)
    g = wl.graph
    rng = np.random.default_rng(4)
    sizes = [0, 1, 2, 5, 13, 20, 32, 9]
    picks = np.concatenate([rng.choice(wl.picks, s) for s in sizes]).astype(np.uint32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    xy = np.stack([picks % g.W, picks // g.W], 1).astype(np.int32)
    no = len(sizes)
    ncell = int((np.diff(off.astype(np.int64)) ** 2).sum())
    for m in (10,):
        st, out, _, err = harness.run(g.row_ptr, g.col, g.w, pick_offsets=off, picks=picks, algo="overlay",
                                      seg=("grid", g.W, g.H, 1, 8, 8), clustered=(m, xy))
        assert st == 0, err[-2000:]
        words = out[ncell:ncell + 2 * no].astype(np.uint64)
        lens = words[0::2] | (words[1::2] << np.uint64(32))
        rts = out[ncell + 2 * no:ncell + 2 * no + len(picks)]
        used = out[ncell + 2 * no + len(picks):]
        el, er, eu = oracle.order_routes_clustered(off, out[:ncell], xy, m, m_max=10)
        assert (lens == el).all() and (rts == er).all() and (used == eu).all()
