"""The library's unchanged HIP kernels and host runtime, run on the CPU by the
test executor (tests/simt_cpu: lanes as threads, emulated wave collectives
and barriers, AddressSanitizer on every buffer), against the oracle.  This
checks the kernels' logic and bounds without a GPU; the GPU tests check the
same paths on the hardware.

Each case runs in its own driver process; the cases start together (the
executor is bound by thread wake-ups, not by arithmetic), and one test
collects every case's verdict."""
import concurrent.futures as cf
import traceback

import numpy as np
import pytest

import oracle
from wgen import make_config

pytestmark = pytest.mark.slow

CASES = []


def case(fn):
    CASES.append(fn)
    return fn


def test_kernels_on_cpu_executor():
    from tests.simt_cpu import harness
    harness.driver(rebuild=True)
    with cf.ThreadPoolExecutor(max_workers=len(CASES)) as ex:
        futs = {fn.__name__: ex.submit(fn, harness) for fn in CASES}
    failed = {}
    for name, f in futs.items():
        try:
            f.result()
        except Exception:
            failed[name] = traceback.format_exc()[-3000:]
    assert not failed, "\n\n".join(f"{k}:\n{v}" for k, v in failed.items())


@case
def case_overlay_order_matrices_tiny(harness):
    wl = make_config("tiny")
    g = wl.graph
    st, out, _, err = harness.run(g.row_ptr, g.col, g.w, pick_offsets=wl.pick_offsets, picks=wl.picks,
                                  algo="overlay", seg=("grid", g.W, g.H, 1, g.W // 3, g.H // 3))
    assert st == 0, err[-2000:]
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (out == exp).all()


@case
def case_overlay_pruned_orders(harness):
    """Target-bounded passes (WR_PRUNE_TO_PICKS) on orders whose picks lie
    close together, with an order of one pick, a duplicate pick and a pick
    shared by two orders: matrices equal the oracle's."""
    from wgen.orders import window_orders
    wl = make_config("medium", side=24, num_orders=1)
    g = wl.graph
    rng = np.random.default_rng(12)
    off, picks = window_orders(rng, g.aisle_adjacent_vertices(), g.W, g.H, 5, 6, 6)
    sizes = list(np.diff(off.astype(np.int64))) + [1, 3]
    picks = np.concatenate([picks, picks[:1], [picks[2], picks[2], picks[7]]]).astype(np.uint32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    st, out, _, err = harness.run(g.row_ptr, g.col, g.w, pick_offsets=off, picks=picks, algo="overlay_prune",
                                  seg=("grid", g.W, g.H, 1, 6, 8))
    assert st == 0, err[-2000:]
    assert (out == oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks)).all()


@case
def case_segmented_rows_and_pred_random_graph(harness):
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


@case
def case_overlay_full_rows_executor(harness):
    """Full rows under the overlay schedule (the tile-blocked read-out):
    sources spread over several 64-source blocks, a source asked for twice
    (a second row group of its block) and a blocked cell (no arcs, only
    itself at 0), with predecessors; rows equal the oracle's."""
    wl = make_config("medium", side=15, num_orders=1)
    g = wl.graph
    rng = np.random.default_rng(8)
    free = np.flatnonzero(np.diff(g.row_ptr.astype(np.int64)) > 0)
    blocked = np.flatnonzero(np.diff(g.row_ptr.astype(np.int64)) == 0)
    src = rng.choice(free, 66, replace=False).astype(np.uint32)
    src = np.concatenate([src, src[[3, 65]], blocked[:1]]).astype(np.uint32)
    st, out, pred, err = harness.run(g.row_ptr, g.col, g.w, sources=src, algo="overlay", pred=True,
                                     seg=("grid", g.W, g.H, 1, 6, 5))
    assert st == 0, err[-2000:]
    d = out.reshape(len(src), g.V)
    p = pred.reshape(len(src), g.V)
    exp = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, src)
    assert (d == exp).all()
    for i, s in enumerate(src):
        assert (p[i] == oracle.canonical_pred(g.row_ptr, g.col, g.w, int(s), exp[i])).all()


@case
def case_order_routes_over_executor_matrices(harness):
    """wr_order_routes (subset programme in LDS) over the library's own
    matrices for orders of 0..12 stops with duplicate picks: lengths and
    orderings equal the oracle's, with every LDS and global access checked."""
    wl = make_config("medium", side=24, num_orders=8)
    g = wl.graph
    rng = np.random.default_rng(3)
    sizes = [0, 1, 2, 3, 5, 12, 4]
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


@case
def case_clustered_routes_over_executor_matrices(harness):
    """wr_order_routes_clustered (K-means in wave 0, the per-cluster and the
    chaining subset programmes) over executor-computed matrices, orders of
    0..13 picks at m = 10 (the largest chaining programme, ten clusters of
    one or two picks): lengths, orderings and cluster counts equal the
    oracle's."""
    wl = make_config("medium", side=24, num_orders=8)
    g = wl.graph
    rng = np.random.default_rng(4)
    sizes = [0, 1, 2, 5, 13]
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


@case
def case_warehouse_loop(harness):
    """wr_wms_run (K-means of the purchase orders, silhouette and area,
    picks with nearest-empty restocking from the racks' shelf masks): the
    final state, the moves, the silhouettes and the areas of every
    iteration equal the oracle's.  An order whose random replacements repeat
    articles (live state in the hash cells), and a small shape with more
    than 16 shelves (32-bit rack masks), four purchase orders of three
    articles in four clusters and fresh parcels per iteration."""
    from oracle import wms
    from wgen.wms import make_wms
    for s in (make_wms(2, 10, 8, 3, 7, 1, 3, 2),
              make_wms(5, 6, 5, 20, 3, 1, 3, 3, po=4, per_po=3, k=4, qty_per_iter=True)):
        st, A, M, sil, area, moves, err = harness.run_wms(s)
        assert st == 0, err[-2000:]
        eA, eM, esil, earea, emv = wms.run(s, 0)
        assert (A[0] == eA).all() and (M[0] == eM).all() and (moves[0] == emv).all()
        assert (sil[0] == esil).all() and (area[0] == earea).all()


@case
def case_server_two_epochs(harness):
    """The streaming server with two resident weight epochs
    (resident_epochs = 2: the scheduler
    thread, row admission, both copies' steps and read-outs, the copy of the
    graph made at the server's start): after a first order, orders arrive one
    every 20 ms with two updates between them; every order's matrix equals
    the oracle's at the weights of the epoch it reports, and the epochs never
    go back."""
    wl = make_config("medium", side=16, num_orders=1)
    g = wl.graph
    rng = np.random.default_rng(12)
    cand = g.aisle_adjacent_vertices()
    picks = np.concatenate([rng.choice(cand, 6, replace=False) for _ in range(6)]).astype(np.uint32)
    off = np.arange(7, dtype=np.uint32) * 6
    ups, weights = [], [g.w.copy()]
    for after in (2, 4):
        arcs = rng.choice(g.E, g.E // 10, replace=False).astype(np.uint32)
        nw = rng.integers(1, 20, len(arcs)).astype(np.uint32)
        ups.append((arcs, nw, after))
        w = weights[-1].copy()
        w[arcs] = nw
        weights.append(w)
    st, out, _, err = harness.run(g.row_ptr, g.col, g.w, pick_offsets=off, picks=picks,
                                  seg=("grid", g.W, g.H, 1, 8, 8), server_gap_ms=20, server_updates=ups)
    assert st == 0, err[-2000:]
    n = len(off) - 1
    epochs = out[-n:].astype(np.int64)
    # orders are solved on the epoch current at their admission, which may
    # come after updates queued behind them (the executor's steps are slow)
    assert (np.diff(epochs) >= 0).all() and epochs[-1] <= 2
    assert epochs[0] == 0 and (epochs[2:] >= 1).all()
    base = 0
    for o in range(n):
        P = int(off[o + 1] - off[o])
        D = out[base:base + P * P].reshape(P, P)
        base += P * P
        pk = picks[off[o]:off[o + 1]]
        exp = oracle.order_matrices(g.row_ptr, g.col, weights[epochs[o]], np.array([0, P], np.uint32), pk)
        assert (D.ravel() == exp).all(), f"order {o} epoch {epochs[o]}"


@case
def case_frontier_rows_random_graph(harness):
    """The push-frontier schedule (wave-aggregated queue appends, pass
    stamps) on a random graph with parallel arcs and self-loops, and on a
    vertex of out-degree above 64 (the aggregation flushes every 64
    targets): rows equal to the oracle's Dijkstra."""
    from tests.helpers import random_csr
    rng = np.random.default_rng(37)
    V = 150
    rp, col, w = random_csr(rng, V, 4 * V, wmax=20)
    # vertex 0 gets 100 more arcs (to every vertex 1..100)
    rows = [list(zip(col[rp[u]:rp[u + 1]], w[rp[u]:rp[u + 1]])) for u in range(V)]
    rows[0] += [(x, int(rng.integers(1, 30))) for x in range(1, 101)]
    rp2 = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.uint32)
    col2 = np.array([x for r in rows for x, _ in r], np.uint32)
    w2 = np.array([y for r in rows for _, y in r], np.uint32)
    src = np.concatenate([[0], rng.choice(np.arange(1, V), 7, replace=False)]).astype(np.uint32)
    st, out, _, err = harness.run(rp2, col2, w2, sources=src, algo="frontier")
    assert st == 0, err[-2000:]
    d = out.reshape(len(src), V)
    for i, s in enumerate(src):
        assert (d[i] == oracle.dijkstra(rp2, col2, w2, int(s))).all(), f"source {s}"
