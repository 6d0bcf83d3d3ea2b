"""GPU parity: every schedule of the HIP path against the CPU oracle,
element by element (integer distances: bit-exact)."""
import numpy as np
import pytest

import oracle
from tests.helpers import random_csr
from wgen import make_config

pytestmark = pytest.mark.gpu
ALGOS = ["segmented", "frontier", "sweep", "edge_b1"]
INF = 0xFFFFFFFF


@pytest.fixture(scope="module")
def ctx(rt):
    return rt.Context(0)


def _graph(rt, ctx, row_ptr, col, w):
    return rt.Graph(ctx, row_ptr, col, w)


@pytest.mark.parametrize("algo", ALGOS + ["edge_b0", "overlay", "auto"])
def test_tiny_order_matrix(rt, ctx, algo):
    wl = make_config("tiny")
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    got = G.order_matrices(wl.pick_offsets, wl.picks, algo=algo)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert got.dtype == np.uint32 and (got == exp).all()
    if algo != "auto":
        assert G.last_run()["algo"] == algo


# (tile vertices, waves): tiles up to 512 vertices run the source-blocked
# kernel, larger ones one source per wave
SCHEDULES = [(256, 8), (512, 16), (1024, 8), (2048, 4)]


@pytest.mark.parametrize("sched", SCHEDULES)
def test_schedules_tiny(rt, ctx, sched):
    wl = make_config("tiny")
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    G.set_schedule(*sched)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (G.order_matrices(wl.pick_offsets, wl.picks, algo="segmented") == exp).all()


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("seed", range(4))
def test_random_graph_sssp(rt, ctx, algo, seed):
    rng = np.random.default_rng(500 + seed)
    V = 300 + 37 * seed
    rp, col, w = random_csr(rng, V, 4 * V, wmax=60, zero_frac=0.1 if seed % 2 else 0.0)
    G = _graph(rt, ctx, rp, col, w)
    if seed >= 2:
        G.set_schedule(*SCHEDULES[seed])
    src = rng.choice(V, 70, replace=False).astype(np.uint32)
    src = np.concatenate([src, src[:5]])            # duplicates
    got = G.sssp(src, algo=algo)
    exp = oracle.dijkstra_multi(rp, col, w, src)
    assert (got == exp).all()


@pytest.mark.parametrize("algo", ALGOS)
def test_pred_matches_canonical(rt, ctx, algo):
    rng = np.random.default_rng(9)
    V = 400
    rp, col, w = random_csr(rng, V, 5 * V, wmax=4)          # many ties
    G = _graph(rt, ctx, rp, col, w)
    src = rng.choice(V, 20, replace=False).astype(np.uint32)
    d, p = G.sssp(src, pred=True, algo=algo)
    for i, s in enumerate(src):
        ed = oracle.dijkstra(rp, col, w, int(s))
        assert (d[i] == ed).all()
        assert (p[i] == oracle.canonical_pred(rp, col, w, int(s), ed)).all()
        assert oracle.certificate(rp, col, w, int(s), d[i], p[i]) == 0


def test_pred_refused_with_zero_weights(rt, ctx):
    rp = np.asarray([0, 1, 2], np.uint32)
    G = _graph(rt, ctx, rp, np.asarray([1, 0], np.uint32), np.asarray([0, 3], np.uint32))
    with pytest.raises(rt.WrError) as ei:
        G.sssp([0], pred=True)
    assert ei.value.name == "WR_E_UNSUPPORTED"
    assert (G.sssp([0]) == np.asarray([[0, 0]], np.uint32)).all()


@pytest.mark.parametrize("tw", [16, 32, 48, 64])
def test_overlay_tile_sizes(rt, ctx, tw):
    """The overlay pass over square grid tiles of several sizes: larger tiles
    have more incoming arcs and exits, so the pass runs with more rows and
    exits per wave; matrices equal the oracle's (tilings beyond the table
    limits are refused, never approximated)."""
    wl = make_config("medium", side=192, num_orders=8)
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, tw, tw)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    try:
        got = G.order_matrices(wl.pick_offsets, wl.picks, algo="overlay")
    except rt.WrError as e:
        assert e.name == "WR_E_UNSUPPORTED" and tw > 32
        pytest.skip(f"{tw}x{tw} tiles exceed the overlay tables")
    assert (got == exp).all()
    again = G.order_matrices(wl.pick_offsets, wl.picks, algo="overlay", graph_capture=False)
    assert (again == exp).all()


def test_overlay_refuses_tiles_with_many_incoming_arcs(rt, ctx):
    """The overlay's exit tables have one column per incoming cross arc, at
    most 64 per tile.  Tile A = {a, b} has 2 ports but 80 incoming cross arcs
    (each of the 40 exits of tile B has an arc to both): the overlay refuses
    the tiling, and the automatic choice falls back to the segmented schedule
    with the oracle's distances."""
    rng = np.random.default_rng(64)
    n = 40
    V = n + 2                       # 0 = a, 1 = b, 2.. = the chain of tile B
    arcs = [(0, 1), (1, 0), (0, 2)]
    for i in range(n):
        v = 2 + i
        arcs += [(v, 0), (v, 1)]
        if i + 1 < n:
            arcs += [(v, v + 1), (v + 1, v)]
    arcs.sort()
    src_v = np.asarray([a for a, _ in arcs], np.int64)
    col = np.asarray([b for _, b in arcs], np.uint32)
    rp = np.zeros(V + 1, np.uint32)
    np.add.at(rp, src_v + 1, 1)
    rp = np.cumsum(rp).astype(np.uint32)
    w = rng.integers(1, 10, len(col)).astype(np.uint32)
    G = _graph(rt, ctx, rp, col, w)
    seg = np.ones(V, np.uint32)
    seg[:2] = 0
    G.set_segments(seg, 2)
    src = np.asarray([0, 5, V - 1], np.uint32)
    exp = oracle.dijkstra_multi(rp, col, w, src)
    with pytest.raises(rt.WrError) as ei:
        G.sssp(src, algo="overlay")
    assert ei.value.name == "WR_E_UNSUPPORTED"
    assert (G.sssp(src, algo="auto") == exp).all()
    assert G.last_run()["algo"] == "segmented"
    assert (G.sssp(src, algo="segmented") == exp).all()


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("seg", ["grid32", "grid_rect", "bfs", "user_map"])
def test_medium_slice_segmented(rt, ctx, seg, sched):
    wl = make_config("medium", side=128, num_orders=12)
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    G.set_schedule(*sched)
    if seg == "grid32":
        G.segment_grid(g.W, g.H, 1, 32, 32)
    elif seg == "grid_rect":
        G.segment_grid(g.W, g.H, 1, 64, 40)          # ragged last row of tiles
    elif seg == "user_map":
        rng = np.random.default_rng(3)
        G.set_segments(rng.integers(0, 7, g.V).astype(np.uint32), 7)   # scattered segments
    got = G.order_matrices(wl.pick_offsets, wl.picks, algo="segmented")
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (got == exp).all()
    info = G.segment_info()
    assert info["tiles"] >= 1
    if seg.startswith("grid") and sched[0] <= 512:
        assert (G.order_matrices(wl.pick_offsets, wl.picks, algo="overlay") == exp).all()


def test_medium_slice_frontier_and_sweep_agree(rt, ctx):
    wl = make_config("medium", side=96, num_orders=6)
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    for algo in ("frontier", "sweep", "segmented"):
        assert (G.order_matrices(wl.pick_offsets, wl.picks, algo=algo) == exp).all(), algo


def test_edge_cases(rt, ctx):
    wl = make_config("tiny")
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    blocked = int(np.flatnonzero(g.blocked.ravel())[0])
    a, b = int(wl.picks[0]), int(wl.picks[1])
    # empty order, duplicates, an order on a blocked (isolated) cell
    off = np.asarray([0, 0, 3, 5, 6], np.uint32)
    picks = np.asarray([a, b, a, blocked, a, blocked], np.uint32)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks)
    for algo in ALGOS:
        got = G.order_matrices(off, picks, algo=algo)
        assert (got == exp).all(), algo
    # isolated source row: 0 at itself, INF elsewhere
    for algo in ALGOS:
        d = G.sssp([blocked], algo=algo)[0]
        assert d[blocked] == 0 and (np.delete(d, blocked) == INF).all()


def test_single_vertex_and_no_arcs(rt, ctx):
    G = _graph(rt, ctx, np.asarray([0, 0], np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    for algo in ALGOS:
        assert (G.sssp([0, 0], algo=algo) == 0).all()


def test_graph_capture_matches_eager(rt, ctx):
    wl = make_config("medium", side=64, num_orders=4)
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 16, 16)
    for algo in ("segmented", "overlay", "frontier"):
        a = G.order_matrices(wl.pick_offsets, wl.picks, algo=algo)
        b = G.order_matrices(wl.pick_offsets, wl.picks, algo=algo, graph_capture=False)
        c = G.order_matrices(wl.pick_offsets, wl.picks, algo=algo)   # replay again
        assert (a == b).all() and (a == c).all()


@pytest.mark.parametrize("algo", ["overlay", "segmented"])
def test_sssp_full_rows_segmented_schedules(rt, ctx, algo):
    wl = make_config("medium", side=80, num_orders=2)
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 16, 16)
    src = np.concatenate([wl.picks[:40], wl.picks[:3]])     # 43 rows, duplicates
    d, p = G.sssp(src, pred=True, algo=algo)
    exp = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, src)
    assert (d == exp).all()
    for i in range(0, len(src), 7):
        assert (p[i] == oracle.canonical_pred(g.row_ptr, g.col, g.w, int(src[i]), exp[i])).all()


def test_device_pointers(rt, ctx):
    import torch
    wl = make_config("medium", side=64, num_orders=5)
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    sizes = np.diff(wl.pick_offsets.astype(np.int64))
    total = int((sizes ** 2).sum())
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    G.order_matrices(wl.pick_offsets, wl.picks, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (got == exp).all()
    src = wl.picks[:7]
    d = torch.empty((7, g.V), dtype=torch.int32, device="cuda")
    G.sssp(src, out=d)
    torch.cuda.synchronize()
    assert (d.cpu().numpy().view(np.uint32) == oracle.dijkstra_multi(g.row_ptr, g.col, g.w, src)).all()


def test_weight_update_epochs(rt, ctx):
    wl = make_config("medium", side=64, num_orders=4)
    g = wl.graph
    G = _graph(rt, ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 32, 32)
    rng = np.random.default_rng(11)
    k = len(g.edge_arc_a) // 20
    pick = rng.choice(len(g.edge_arc_a), k, replace=False)
    neww = (g.edge_base_w[pick] + rng.integers(0, 21, k)).astype(np.uint32)
    arcs = np.concatenate([g.edge_arc_a[pick], g.edge_arc_b[pick]]).astype(np.uint32)
    vals = np.concatenate([neww, neww])
    ep = G.update_weights(arcs, vals)
    assert ep == 1
    w2 = g.w.copy()
    w2[arcs] = vals
    exp = oracle.order_matrices(g.row_ptr, g.col, w2, wl.pick_offsets, wl.picks)
    for algo in ("segmented", "overlay", "frontier", "sweep", "edge_b1"):
        assert (G.order_matrices(wl.pick_offsets, wl.picks, algo=algo) == exp).all(), algo
    # a second update: the overlay tables follow the new epoch
    w3 = w2.copy()
    w3[arcs] = np.maximum(vals, 2) - 1
    assert G.update_weights(arcs, w3[arcs]) == 2
    exp3 = oracle.order_matrices(g.row_ptr, g.col, w3, wl.pick_offsets, wl.picks)
    for algo in ("overlay", "segmented"):
        assert (G.order_matrices(wl.pick_offsets, wl.picks, algo=algo) == exp3).all(), algo


def test_overlay_chunks_under_small_budget(rt):
    """A memory budget too small for every source block at once: the batch
    is solved chunk by chunk, and the matrices stay exact."""
    wl = make_config("medium", side=128, num_orders=16)
    g = wl.graph
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    for budget_mb in (66, 68, 70, 72, 76, 80, 96):
        try:
            ctx = rt.Context(0, budget_mb << 20)
            G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
            G.set_schedule(512, 8, 0)
            G.segment_grid(g.W, g.H, 1, 24, 20)
            got = G.order_matrices(wl.pick_offsets, wl.picks, algo="overlay")
        except rt.WrError as e:
            assert e.name == "WR_E_NOMEM"
            continue
        if G.last_run()["chunks"] > 1:
            assert (got == exp).all()
            return
    pytest.fail("no budget produced a chunked run")


def test_overlay_back_to_back_calls(rt, ctx):
    """Consecutive overlay calls on one graph reuse the per-call state (reset
    after each call): batches of growing and shrinking source counts, with
    a weight update in between, all stay exact."""
    wl = make_config("medium", side=96, num_orders=24)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 12, 10)
    off, picks = wl.pick_offsets, wl.picks
    w = g.w.copy()
    rng = np.random.default_rng(5)
    for n_orders in (24, 3, 17, 1, 24):
        o_off = off[:n_orders + 1]
        o_picks = picks[:int(o_off[-1])]
        got = G.order_matrices(o_off, o_picks, algo="overlay")
        exp = oracle.order_matrices(g.row_ptr, g.col, w, o_off, o_picks)
        assert (got == exp).all(), f"{n_orders} orders"
        if n_orders == 17:
            arcs = rng.choice(g.E, g.E // 10, replace=False).astype(np.uint32)
            neww = rng.integers(1, 25, len(arcs)).astype(np.uint32)
            G.update_weights(arcs, neww)
            w[arcs] = neww
