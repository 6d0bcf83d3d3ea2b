"""GPU tests of the continuous-batching server and the autotuner against the
CPU oracle: every order's matrix is exact whether it is solved alone or in
a mix, results are pinned to the weight epoch current at admission, a
request that can never fit the memory budget fails alone, and every
autotuner choice gives the default's bits."""
import time

import numpy as np
import pytest

import oracle
from wgen import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(rt):
    return rt.Context(0)


def _small(rt, ctx, side=48, orders=12):
    wl = make_config("medium", side=side, num_orders=orders)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 12, 10)
    return wl, G


def _orders(wl):
    off = wl.pick_offsets
    return [wl.picks[off[o]:off[o + 1]].copy() for o in range(len(off) - 1)]


def _expect(g, picks, w=None):
    off = np.array([0, len(picks)], dtype=np.uint32)
    P = len(picks)
    return oracle.order_matrices(g.row_ptr, g.col, g.w if w is None else w, off, picks).reshape(P, P)


def _wait(srv, tickets, timeout=120.0):
    res = {}
    t_end = time.time() + timeout
    while len(res) < len(tickets):
        assert time.time() < t_end, "server did not finish in time"
        for t in tickets:
            if t in res:
                continue
            m, info = srv.poll(t)
            if m is not None:
                res[t] = (m, info)
        time.sleep(0.002)
    return res


def test_server_alone_equals_mix(rt, ctx):
    wl, G = _small(rt, ctx)
    g = wl.graph
    orders = _orders(wl)
    srv = rt.Server(G, max_source_slots=256)
    try:
        alone = []
        for pk in orders[:4]:
            t = srv.submit(pk)
            srv.drain()
            alone.append(_wait(srv, [t])[t][0])
        tickets = [srv.submit(pk) for pk in orders]
        got = _wait(srv, tickets)
        for i, pk in enumerate(orders):
            m, info = got[tickets[i]]
            exp = _expect(g, pk)
            assert (m == exp).all(), f"order {i}"
            assert info["status"] == 0 and info["P"] == len(pk)
            assert info["t_arrive"] <= info["t_admit"] <= info["t_done"]
            if i < 4:
                assert (alone[i] == m).all()
        st = srv.stats()
        assert st["completed"] == 4 + len(orders) and st["failed"] == 0
        assert st["p99_ms"] >= st["p50_ms"] > 0 and st["throughput_per_s"] > 0
    finally:
        srv.close()


def test_server_empty_order_and_duplicates(rt, ctx):
    wl, G = _small(rt, ctx, side=32, orders=2)
    g = wl.graph
    srv = rt.Server(G)
    try:
        t0 = srv.submit(np.zeros(0, dtype=np.uint32))
        pk = np.array([wl.picks[0], wl.picks[1], wl.picks[0]], dtype=np.uint32)
        t1 = srv.submit(pk)
        res = _wait(srv, [t0, t1])
        assert res[t0][0].shape == (0, 0)
        m = res[t1][0]
        assert (m == _expect(g, pk)).all()
        assert m[0, 2] == 0 and (m[0] == m[2]).all()
    finally:
        srv.close()


@pytest.mark.parametrize("resident", [1, 2])
def test_server_weight_epochs(rt, ctx, resident):
    wl, G = _small(rt, ctx, side=40, orders=6)
    g = wl.graph
    orders = _orders(wl)
    srv = rt.Server(G, resident_epochs=resident)
    try:
        t_before = [srv.submit(pk) for pk in orders[:3]]
        first = _wait(srv, t_before)
        rng = np.random.default_rng(77)
        arcs = rng.choice(g.E, g.E // 20, replace=False).astype(np.uint32)
        new_w = rng.integers(1, 30, len(arcs)).astype(np.uint32)
        srv.update_weights(arcs, new_w)
        w2 = g.w.copy()
        w2[arcs] = new_w
        t_after = [srv.submit(pk) for pk in orders]
        after = _wait(srv, t_after)
        e0 = {first[t][1]["epoch"] for t in t_before}
        e1 = {after[t][1]["epoch"] for t in t_after}
        assert len(e0) == 1 and len(e1) == 1 and min(e1) == max(e0) + 1
        for i, t in enumerate(t_before):
            assert (first[t][0] == _expect(g, orders[i])).all()
        for i, t in enumerate(t_after):
            assert (after[t][0] == _expect(g, orders[i], w2)).all()
    finally:
        srv.close()


def test_server_memory_admission(rt, ctx):
    wl, G = _small(rt, ctx, side=32, orders=2)
    srv = rt.Server(G, mem_budget_bytes=1)
    try:
        t_empty = srv.submit(np.zeros(0, dtype=np.uint32))
        t_big = srv.submit(wl.picks[:8])
        m, _ = _wait(srv, [t_empty])[t_empty]
        assert m.shape == (0, 0)
        t_end = time.time() + 60
        while True:
            try:
                m, info = srv.poll(t_big)
            except rt.WrError as e:
                assert e.name == "WR_E_NOMEM"
                break
            assert m is None and time.time() < t_end
            time.sleep(0.002)
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 1
    finally:
        srv.close()


def test_server_rejects_bad_input(rt, ctx):
    wl, G = _small(rt, ctx, side=24, orders=1)
    srv = rt.Server(G)
    try:
        with pytest.raises(rt.WrError) as e:
            srv.submit(np.array([wl.graph.V], dtype=np.uint32))
        assert e.value.name == "WR_E_INVALID"
        with pytest.raises(rt.WrError):
            srv.update_weights(np.array([wl.graph.E], dtype=np.uint32), np.array([1], dtype=np.uint32))
    finally:
        srv.close()


def test_autotune_identical_results(rt, ctx, tmp_path):
    wl, G = _small(rt, ctx, side=48, orders=6)
    g = wl.graph
    exp = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (G.order_matrices(wl.pick_offsets, wl.picks) == exp).all()
    cache = tmp_path / "tune.json"
    G.autotune(sources_hint=64, cache_path=str(cache))
    assert cache.exists()
    assert (G.order_matrices(wl.pick_offsets, wl.picks) == exp).all()
    # a second graph of the same structure reads the cache and gets the same bits
    G2 = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G2.segment_grid(g.W, g.H, 1, 12, 10)
    t = time.time()
    G2.autotune(sources_hint=64, cache_path=str(cache))
    assert time.time() - t < 5.0
    assert (G2.order_matrices(wl.pick_offsets, wl.picks) == exp).all()


def test_server_admits_while_others_relax(rt, ctx):
    """Continuous batching: an order that arrives while another is relaxing is
    admitted before that one finishes (step batching could only admit it
    afterwards), and both results stay exact."""
    wl = make_config("medium", side=256, num_orders=24)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 24, 20)
    G.set_schedule(512, 8, 0)
    orders = _orders(wl)
    srv = rt.Server(G, passes_per_step=2)
    try:
        tickets = []
        for pk in orders:
            tickets.append(srv.submit(pk))
            time.sleep(0.0005)
        res = _wait(srv, tickets)
        info = [res[t][1] for t in tickets]
        overlap = any(info[i]["t_admit"] < info[j]["t_admit"] < info[i]["t_done"]
                      for i in range(len(info)) for j in range(len(info)))
        assert overlap, "no order was admitted while another was in flight"
        for i, t in enumerate(tickets):
            assert (res[t][0] == _expect(g, orders[i])).all(), f"order {i}"
        assert srv.stats()["max_inflight_requests"] > 1
    finally:
        srv.close()


def _expect_many(g, orders, w):
    """Oracle matrices of several orders at weights w (one call)."""
    off = np.concatenate([[0], np.cumsum([len(o) for o in orders])]).astype(np.uint32)
    flat = oracle.order_matrices(g.row_ptr, g.col, w, off, np.concatenate(orders).astype(np.uint32))
    res, base = [], 0
    for o in orders:
        P = len(o)
        res.append(flat[base:base + P * P].reshape(P, P))
        base += P * P
    return res


def test_server_ticks_mid_flight_full_graph(rt, ctx):
    """Two weight epochs resident, on the full serving graph (3 x 1024^2 with
    lifts): orders in flight when a congestion tick (1 % of the arcs) arrives
    finish on their epoch while the orders after it run on the new one, and a
    second tick right after waits for a copy with nothing in flight; every
    order's matrix equals the oracle's at its own epoch's weights."""
    from bench import graph_for
    wl = make_config("serving")
    g = wl.graph
    G, _ = graph_for(rt, ctx, wl, tune=False)
    rng = np.random.default_rng(91)
    cand = g.aisle_adjacent_vertices()
    pick = lambda P: cand[rng.choice(len(cand), P, replace=False)].astype(np.uint32)
    batches = [[pick(96) for _ in range(3)], [pick(8) for _ in range(3)], [pick(6) for _ in range(2)]]
    weights = [g.w.copy()]
    srv = rt.Server(G, resident_epochs=2)
    try:
        # the server is up (its rows built) before the batches arrive, and
        # its epoch before any update is that of a 0-pick order
        e0 = _wait(srv, [srv.submit(np.zeros(0, np.uint32))])
        e0 = next(iter(e0.values()))[1]["epoch"]
        _wait(srv, [srv.submit(pick(2))])
        tickets = [[srv.submit(o) for o in batches[0]]]
        time.sleep(0.01)
        for k in (1, 2):
            arcs = rng.choice(g.E, g.E // 100, replace=False).astype(np.uint32)
            new_w = rng.integers(1, 11, len(arcs)).astype(np.uint32)
            srv.update_weights(arcs, new_w)
            w = weights[-1].copy()
            w[arcs] = new_w
            weights.append(w)
            tickets.append([srv.submit(o) for o in batches[k]])
        res = _wait(srv, [t for ts in tickets for t in ts], timeout=300.0)
    finally:
        srv.close()
    e_base = e0
    infos = {t: res[t][1] for ts in tickets for t in ts}
    # every order on one of the three epochs, and not older than its submission
    for k, ts in enumerate(tickets):
        for t in ts:
            assert e_base <= infos[t]["epoch"] <= e_base + 2
            assert infos[t]["epoch"] >= e_base + (k if k == 0 else 1)
    # both epochs in flight at once: an order of the first epoch finished
    # after an order of a later epoch had been admitted
    first = [infos[t] for t in tickets[0] if infos[t]["epoch"] == e_base]
    later = [i for i in infos.values() if i["epoch"] > e_base]
    assert first and later
    assert max(i["t_done"] for i in first) > min(i["t_admit"] for i in later)
    for k, ts in enumerate(tickets):
        for e in range(3):
            sel = [i for i, t in enumerate(ts) if infos[t]["epoch"] == e_base + e]
            if not sel:
                continue
            exp = _expect_many(g, [batches[k][i] for i in sel], weights[e])
            for i, E in zip(sel, exp):
                assert (res[ts[i]][0] == E).all(), f"batch {k} order {i} epoch {e}"
