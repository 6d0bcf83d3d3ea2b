"""Pins for the CPU oracle: every check here compares it with something other
than itself (brute-force enumeration, closed forms, scipy's Dijkstra, planted
mistakes that the certificate must catch)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra as sp_dijkstra

import oracle
from oracle.brute import all_pairs_by_enumeration
from oracle.closed_forms import manhattan, rack_distance
from tests.helpers import random_csr, csr_arcs
from wgen import build_grid_graph, make_config, rack_layout

INF = oracle.INF
pytestmark = pytest.mark.filterwarnings("ignore")


def _scipy_rows(row_ptr, col, w, sources):
    """scipy csgraph Dijkstra; parallel arcs are reduced to their minimum."""
    V = len(row_ptr) - 1
    rows = np.repeat(np.arange(V), np.diff(row_ptr.astype(np.int64)))
    keep = rows != col
    # csgraph treats explicit zeros as absent arcs; shift weights by +1 and
    # rebuild exact distances through a tiny epsilon-free trick is not
    # possible, so only use positive-weight graphs here
    assert (w[keep] > 0).all()
    m = {}
    for a, b, c in zip(rows[keep], col[keep], w[keep]):
        k = (int(a), int(b))
        m[k] = min(m.get(k, 1 << 62), int(c))
    if m:
        r, c = zip(*m.keys())
        data = list(m.values())
    else:
        r, c, data = [], [], []
    G = sp.csr_matrix((np.asarray(data, float), (r, c)), shape=(V, V))
    D = sp_dijkstra(G, indices=np.asarray(sources))
    out = np.where(np.isfinite(D), D, INF).astype(np.uint64)
    return out


@pytest.mark.parametrize("seed", range(40))
def test_dijkstra_and_bf_match_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    V = int(rng.integers(1, 10))
    E = int(rng.integers(0, 3 * V + 1))
    rp, col, w = random_csr(rng, V, E, wmax=7, zero_frac=0.25 if seed % 2 else 0.0)
    D = all_pairs_by_enumeration(V, csr_arcs(rp, col, w))
    for s in range(V):
        d = oracle.dijkstra(rp, col, w, s)
        b, _, st = oracle.bellman_ford(rp, col, w, s)
        assert st == 0
        assert d.tolist() == D[s], (s, d, D[s])
        assert b.tolist() == D[s]
        assert oracle.certificate(rp, col, w, s, d) == 0


def test_obstacle_free_grid_is_manhattan():
    for c in (1, 4):
        W, H = 13, 9
        g = build_grid_graph(W, H, range(H), c, c, np.random.default_rng(0))
        assert not g.blocked.any()
        for s in [0, 5, W * 4 + 6, W * H - 1]:
            d = oracle.dijkstra(g.row_ptr, g.col, g.w, s)
            sx, sy = s % W, s // W
            exp = [manhattan(sx, sy, v % W, v // W, c) for v in range(W * H)]
            assert d.tolist() == exp


@pytest.mark.parametrize("c", [1, 3])
def test_tiny_rack_layout_closed_form(c):
    rows = [0, 19, 39]
    g = build_grid_graph(20, 40, rows, c, c, np.random.default_rng(0))
    aisle = [(x, y) for y in range(40) for x in range(20)
             if not g.blocked[y, x] and x % 3 != 2]
    src = np.asarray([y * 20 + x for x, y in aisle], dtype=np.uint32)
    D = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, src)
    bad = 0
    for i, (x1, y1) in enumerate(aisle):
        for (x2, y2) in aisle:
            if D[i, y2 * 20 + x2] != rack_distance(x1, y1, x2, y2, rows, c):
                bad += 1
    assert bad == 0


def test_larger_rack_layout_closed_form_sampled():
    rows = [0, 32, 64, 95]
    W, H = 64, 96
    g = build_grid_graph(W, H, rows, 2, 2, np.random.default_rng(0))
    rng = np.random.default_rng(5)
    aisle = np.asarray([y * W + x for y in range(H) for x in range(W)
                        if not g.blocked[y, x] and x % 3 != 2])
    src = aisle[rng.choice(len(aisle), 40, replace=False)].astype(np.uint32)
    D = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, src)
    for i, s in enumerate(src):
        x1, y1 = int(s) % W, int(s) // W
        for t in aisle:
            x2, y2 = int(t) % W, int(t) // W
            assert D[i, t] == rack_distance(x1, y1, x2, y2, rows, 2)


def test_blocked_cells_unreachable_and_isolated():
    wl = make_config("tiny")
    g = wl.graph
    d = oracle.dijkstra(g.row_ptr, g.col, g.w, int(wl.picks[0]))
    blocked = np.flatnonzero(g.blocked.ravel())
    assert (d[blocked] == INF).all()
    free = np.flatnonzero(~g.blocked.ravel())
    assert (d[free] != INF).all()
    # a source on a blocked cell reaches only itself
    d2 = oracle.dijkstra(g.row_ptr, g.col, g.w, int(blocked[0]))
    assert d2[blocked[0]] == 0 and (np.delete(d2, blocked[0]) == INF).all()


@pytest.mark.parametrize("seed", range(6))
def test_matches_scipy_on_random_graphs(seed):
    rng = np.random.default_rng(77 + seed)
    V = 300
    rp, col, w = random_csr(rng, V, 1200, wmax=50)
    src = rng.choice(V, 12, replace=False).astype(np.uint32)
    D = oracle.dijkstra_multi(rp, col, w, src)
    ref = _scipy_rows(rp, col, w, src)
    assert (D.astype(np.uint64) == ref).all()
    for i, s in enumerate(src):
        b, _, st = oracle.bellman_ford(rp, col, w, int(s))
        assert st == 0 and (b == D[i]).all()


def test_matches_scipy_on_medium_sample():
    wl = make_config("medium")
    g = wl.graph
    src = wl.picks[:6]
    D = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, src)
    ref = _scipy_rows(g.row_ptr, g.col, g.w, src)
    assert (D.astype(np.uint64) == ref).all()


def test_bellman_ford_round_cap_is_hop_depth():
    # a directed path 0->1->...->V-1 needs exactly V-1 changing rounds
    V = 25
    rp = np.arange(V + 1, dtype=np.uint32)
    rp[-1] = V - 1
    col = np.arange(1, V, dtype=np.uint32)
    w = np.full(V - 1, 3, dtype=np.uint32)
    d, rounds, st = oracle.bellman_ford(rp, col, w, 0)
    assert st == 0 and rounds == V - 1
    assert d.tolist() == [3 * i for i in range(V)]
    # with a cap below the hop depth the run reports that it was cut short
    d, rounds, st = oracle.bellman_ford(rp, col, w, 0, max_rounds=5)
    assert st == 4 and rounds == 5


def _brute_pred(V, arcs, src, d):
    pred = [-1] * V
    for v in range(V):
        if v == src or d[v] == INF:
            continue
        cands = [u for (u, x, ww) in arcs if x == v and d[u] != INF and d[u] + ww == d[v]]
        pred[v] = min(cands)
    return pred


@pytest.mark.parametrize("seed", range(20))
def test_canonical_pred_definition(seed):
    rng = np.random.default_rng(4000 + seed)
    V = int(rng.integers(2, 30))
    rp, col, w = random_csr(rng, V, 4 * V, wmax=4)
    arcs = list(csr_arcs(rp, col, w))
    for s in range(min(V, 5)):
        d = oracle.dijkstra(rp, col, w, s)
        p = oracle.canonical_pred(rp, col, w, s, d)
        assert p.tolist() == _brute_pred(V, arcs, s, d.tolist())
        assert oracle.certificate(rp, col, w, s, d, p) == 0


def test_certificate_catches_planted_mistakes():
    wl = make_config("tiny")
    g = wl.graph
    s = int(wl.picks[3])
    d = oracle.dijkstra(g.row_ptr, g.col, g.w, s)
    p = oracle.canonical_pred(g.row_ptr, g.col, g.w, s, d)
    assert oracle.certificate(g.row_ptr, g.col, g.w, s, d, p) == 0
    free = np.flatnonzero(d != INF)
    far = int(free[np.argmax(d[free])])
    mid = int(free[len(free) // 2])
    bad = d.copy(); bad[s] = 1
    assert oracle.certificate(g.row_ptr, g.col, g.w, s, bad) != 0
    bad = d.copy(); bad[mid] += 1           # too long: some in-arc is infeasible
    assert oracle.certificate(g.row_ptr, g.col, g.w, s, bad) == 11
    bad = d.copy(); bad[far] -= 1           # too short: not the length of a path
    assert oracle.certificate(g.row_ptr, g.col, g.w, s, bad) == 12
    bad = d.copy(); bad[mid] = INF          # dropped vertex
    assert oracle.certificate(g.row_ptr, g.col, g.w, s, bad) != 0
    bp = p.copy(); bp[mid] = s if p[mid] != s else -1   # non-tight predecessor
    assert oracle.certificate(g.row_ptr, g.col, g.w, s, d, bp) in (21, 22)
    bp = p.copy(); bp[s] = 0
    assert oracle.certificate(g.row_ptr, g.col, g.w, s, d, bp) == 20


def test_certificate_rows_flags_each_planted_row():
    # the parallel form checks every row on its own: planted mistakes in
    # some rows of a batch are reported on exactly those rows, with the
    # single-row codes
    wl = make_config("tiny")
    g = wl.graph
    src = np.unique(wl.picks)
    d = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, src)
    p = np.stack([oracle.canonical_pred(g.row_ptr, g.col, g.w, int(s), d[i]) for i, s in enumerate(src)])
    assert (oracle.certificate_rows(g.row_ptr, g.col, g.w, src, d, p) == 0).all()
    bad = d.copy()
    free = np.flatnonzero(d[1] != INF)
    bad[1, free[len(free) // 2]] += 1
    bad[4, int(src[4])] = 1
    far = int(free[np.argmax(d[6][free])])
    bad[6, far] -= 1
    rc = oracle.certificate_rows(g.row_ptr, g.col, g.w, src, bad, nthreads=3)
    exp = [oracle.certificate(g.row_ptr, g.col, g.w, int(s), bad[i]) for i, s in enumerate(src)]
    assert rc.tolist() == exp
    assert [i for i in range(len(src)) if rc[i]] == [1, 4, 6]
    # rows paired with the wrong source fail
    assert (oracle.certificate_rows(g.row_ptr, g.col, g.w, src[::-1].copy(), d) != 0).all()


def test_certificate_catches_pred_cycle():
    # two vertices joined by zero-weight arcs, both at distance 1 from 0
    rp = np.asarray([0, 2, 4, 6], dtype=np.uint32)
    col = np.asarray([1, 2, 0, 2, 0, 1], dtype=np.uint32)
    w = np.asarray([1, 1, 1, 0, 1, 0], dtype=np.uint32)
    d = oracle.dijkstra(rp, col, w, 0)
    assert d.tolist() == [0, 1, 1]
    assert oracle.certificate(rp, col, w, 0, d, np.asarray([-1, 2, 1], np.int32)) == 23
    assert oracle.certificate(rp, col, w, 0, d, np.asarray([-1, 0, 0], np.int32)) == 0


def test_order_matrix_properties():
    wl = make_config("medium", num_orders=6)
    g = wl.graph
    M = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    off = wl.pick_offsets
    base = 0
    for o in range(len(off) - 1):
        pk = wl.picks[off[o]:off[o + 1]]
        P = len(pk)
        D = M[base:base + P * P].reshape(P, P).astype(np.int64)
        base += P * P
        assert (np.diag(D) == 0).all()
        assert (D == D.T).all()                      # symmetric weights
        # metric closure: D[i][j] <= D[i][k] + D[k][j]
        assert (D[:, None, :] <= D[:, :, None] + D[None, :, :]).all()
        rows = oracle.dijkstra_multi(g.row_ptr, g.col, g.w, pk[:2])
        assert (D[:2] == rows[:, pk]).all()


def test_order_matrix_duplicates_and_empty():
    wl = make_config("tiny")
    g = wl.graph
    a, b = int(wl.picks[0]), int(wl.picks[1])
    off = np.asarray([0, 3, 3, 4], dtype=np.uint32)   # 3 picks, empty, 1 pick
    picks = np.asarray([a, b, a, b], dtype=np.uint32)
    M = oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks)
    assert len(M) == 9 + 0 + 1
    D = M[:9].reshape(3, 3)
    assert D[0, 2] == 0 and D[2, 0] == 0
    assert (D[0] == D[2]).all() and (D[:, 0] == D[:, 2]).all()
    assert M[9] == 0


def test_validate_csr_rules():
    rp = np.asarray([0, 1, 2], np.uint32)
    col = np.asarray([1, 0], np.uint32)
    w = np.asarray([5, 5], np.uint32)
    assert oracle.validate_csr(rp, col, w) == 0
    assert oracle.validate_csr(np.asarray([0, 1, 3], np.uint32), col, w) == 1   # row_ptr[V] != E
    assert oracle.validate_csr(np.asarray([0, 2, 1], np.uint32), col, w) == 1   # decreasing
    assert oracle.validate_csr(rp, np.asarray([1, 2], np.uint32), w) == 1       # col >= V
    big = np.asarray([0xFFFFFFFF, 1], np.uint32)
    assert oracle.validate_csr(rp, col, big) == 2                              # overflow
    # bound uses incident vertices: 3 incident vertices, max_w * 2 >= INF
    rp3 = np.asarray([0, 1, 2, 2, 2], np.uint32)
    col3 = np.asarray([1, 2], np.uint32)
    assert oracle.validate_csr(rp3, col3, np.asarray([0x80000000, 1], np.uint32)) == 2
    assert oracle.validate_csr(rp3, col3, np.asarray([0x7FFFFFFF, 1], np.uint32)) == 0


def test_generator_counts_match_layout_reading():
    wl = make_config("tiny")
    g = wl.graph
    assert (g.V, g.E) == (800, 1724)
    assert len(g.free_vertices()) == 578
    assert len(g.aisle_adjacent_vertices()) == 462
    wl2 = make_config("medium", num_orders=1)
    assert (wl2.graph.V, wl2.graph.E) == (262144, 536188)
    assert len(wl2.graph.free_vertices()) == 177994
    assert len(wl2.graph.aisle_adjacent_vertices()) == 171190


def _golden(name):
    import os
    return os.path.join(os.path.dirname(__file__), "golden", name)


def test_tiny_golden_matrix_is_stable():
    """The stored matrix was written from the oracle; a change in the
    generator recipe or the oracle's arithmetic shows up here."""
    lines = [l for l in open(_golden("tiny_order_matrix.txt")) if not l.startswith("#")]
    picks = [int(x) for x in lines[0].split()[1:]]
    D = np.asarray([[int(x) for x in l.split()] for l in lines[1:]])
    wl = make_config("tiny")
    assert picks == wl.picks.tolist()
    g = wl.graph
    M = oracle.order_matrices(g.row_ptr, g.col, g.w, wl.pick_offsets, wl.picks)
    assert (M.reshape(8, 8) == D).all()


def test_paper_printed_launch_arithmetic():
    vals = {}
    for l in open(_golden("paper_numbers.txt")):
        l = l.split("#")[0].split()
        if l:
            vals[l[0]] = float(l[1])
    E = int(vals["bf_edges"])
    assert -(-E // int(vals["threads_per_block"])) == vals["blocks_per_round"]
    # the printed MTEPS counts (V-1) full rounds of E edges over the run
    V = int(vals["bf_vertices"])
    mteps = (V - 1) * E / (vals["bf_time_ms"] * 1e-3) / 1e6
    assert abs(mteps - vals["bf_mteps"]) / vals["bf_mteps"] < 0.01
    import math
    assert math.factorial(9) * 8 == vals["perm_limit"]


def test_generators_are_deterministic():
    a = make_config("medium", num_orders=4)
    b = make_config("medium", num_orders=4)
    assert (a.graph.w == b.graph.w).all() and (a.picks == b.picks).all()
    c = make_config("medium", num_orders=4, rep=1)
    assert not (a.graph.w == c.graph.w).all()
    # picks are distinct within an order and aisle-adjacent
    adj = set(a.graph.aisle_adjacent_vertices().tolist())
    for o in range(4):
        pk = a.picks[a.pick_offsets[o]:a.pick_offsets[o + 1]].tolist()
        assert len(set(pk)) == len(pk) and set(pk) <= adj


# ----------------------------------------------------------- optimal routes
def _route_cases():
    """Matrices that expose plausible mistakes: asymmetric entries (a
    transposed step), heavy ties (the tie-break), INF entries (saturation),
    and metric closures of random points (the hot path's matrices)."""
    rng = np.random.default_rng(11)
    cases = []
    for n in range(1, 8):
        cases.append(rng.integers(0, 50, (n, n)))                    # asymmetric
        cases.append(rng.integers(0, 3, (n, n)))                     # many ties
        m = rng.integers(1, 40, (n, n))
        m[rng.random((n, n)) < 0.3] = INF                            # unreachable steps
        cases.append(m)
        pts = rng.integers(0, 20, (n, 2))
        cases.append(np.abs(pts[:, None, :] - pts[None, :, :]).sum(-1))   # L1 metric
    for n in range(3, 8):
        # one stop cut off from the rest: every ordering is infinite, while
        # paths among the other stops stay finite (the tie-break must not
        # follow them)
        m = rng.integers(1, 40, (n, n))
        k = int(rng.integers(0, n))
        m[k, :] = INF
        m[:, k] = INF
        cases.append(m)
    for m in cases:
        np.fill_diagonal(m, 0)
    return [m.astype(np.uint32) for m in cases]


def test_route_matches_enumeration():
    from oracle.brute import route_by_enumeration
    for D in _route_cases():
        cost, r = oracle.route(D)
        best, p = route_by_enumeration(D.tolist())
        assert cost == (oracle.ROUTE_INF if best is None else best), D
        assert r.tolist() == p, D


def test_route_closed_forms():
    # stops on a line: the best open route sweeps from one end to the other,
    # length max - min, visiting the stops in coordinate order
    rng = np.random.default_rng(12)
    for n in (2, 5, 9, 13):
        x = rng.choice(1000, n, replace=False)
        D = np.abs(x[:, None] - x[None, :]).astype(np.uint32)
        cost, r = oracle.route(D)
        assert cost == x.max() - x.min()
        xs = x[r]
        assert (np.diff(xs) > 0).all() or (np.diff(xs) < 0).all()
        # lexicographically smallest of the two sweeps
        asc, desc = np.argsort(x), np.argsort(-x)
        assert r.tolist() == min(asc.tolist(), desc.tolist())
    # degenerate sizes and an infeasible matrix
    assert oracle.route(np.zeros((0, 0), np.uint32))[0] == 0
    c, r = oracle.route(np.zeros((1, 1), np.uint32))
    assert c == 0 and r.tolist() == [0]
    c, r = oracle.route(np.array([[0, 7], [3, 0]], np.uint32))
    assert c == 3 and r.tolist() == [1, 0]
    D = np.full((4, 4), INF, np.uint32)
    np.fill_diagonal(D, 0)
    c, r = oracle.route(D)
    assert c == oracle.ROUTE_INF and r.tolist() == [0, 1, 2, 3]


def test_order_routes_batches_orders():
    mats = _route_cases()[:12]
    sizes = [m.shape[0] for m in mats]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    cost, rt = oracle.order_routes(off, np.concatenate([m.ravel() for m in mats]))
    for o, m in enumerate(mats):
        c, r = oracle.route(m)
        assert cost[o] == c and rt[off[o]:off[o + 1]].tolist() == r.tolist()


# ------------------------------------------------- cluster-decomposed routes
def test_theorem_counts_match_paper():
    """The printed costs of the theorem (m!2^(m-1) undirected chains plus
    n_j!/2 undirected routes inside each of the m clusters) from the
    candidates the oracle itself compares: its chaining enumeration counts
    m!2^m directed chains and its route enumeration n_j! directed orderings,
    each pair of travel directions making one undirected route."""
    import math
    vals = {}
    for l in open(_golden("paper_numbers.txt")):
        l = l.split("#")[0].split()
        if l:
            vals[l[0]] = int(float(l[1]))
    for key, n, m in (("thm_n12_m2", 12, 2), ("thm_n12_m3", 12, 3), ("thm_n12_m4", 12, 4), ("thm_n15_m3", 15, 3)):
        k = n // m
        D = np.zeros((n, n), np.uint32)
        pieces = [list(range(c * k, (c + 1) * k)) for c in range(m)]
        _, chain, n_chains = oracle.chain_routes(pieces, D)
        assert sorted(chain.tolist()) == list(range(n))
        assert n_chains == math.factorial(m) * 2 ** m
        inner = 0
        for p in pieces:
            _, _, n_orderings = oracle.route_enumerate(D[np.ix_(p, p)])
            assert n_orderings == math.factorial(len(p))
            inner += n_orderings // 2
        assert n_chains // 2 + inner == vals[key], key


def test_route_held_karp_matches_c_enumeration():
    """The subset programme against the second, independent method (every
    ordering in C) at the sizes the GPU serves, up to 10 stops (and one of
    11): lengths and the lexicographic tie-break."""
    rng = np.random.default_rng(21)
    for n in (8, 9, 10):
        for kind in range(4):
            if kind == 0:
                D = rng.integers(0, 60, (n, n))
            elif kind == 1:
                D = rng.integers(0, 3, (n, n))
            elif kind == 2:
                D = rng.integers(1, 40, (n, n))
                D[rng.random((n, n)) < 0.35] = INF
            else:
                pts = rng.integers(0, 12, (n, 2))
                D = np.abs(pts[:, None, :] - pts[None, :, :]).sum(-1)
            if n == 9 and kind == 2:
                # a stop cut off from the rest: every ordering infinite
                D[n // 2, :] = INF
                D[:, n // 2] = INF
            D = D.astype(np.uint32)
            np.fill_diagonal(D, 0)
            c1, r1 = oracle.route(D)
            c2, r2, cnt = oracle.route_enumerate(D)
            assert c1 == c2 and r1.tolist() == r2.tolist(), (n, kind)
            import math
            assert cnt == math.factorial(n)
    D = rng.integers(0, 4, (11, 11)).astype(np.uint32)
    np.fill_diagonal(D, 0)
    c1, r1 = oracle.route(D)
    c2, r2, _ = oracle.route_enumerate(D)
    assert c1 == c2 and r1.tolist() == r2.tolist()


def test_route_c_enumeration_matches_python():
    """The C enumeration against the pure-Python one (itertools) on the
    small case families, INF steps and ties included."""
    from oracle.brute import route_by_enumeration
    for D in _route_cases():
        c, r, _ = oracle.route_enumerate(D)
        best, p = route_by_enumeration(D.tolist())
        assert c == (oracle.ROUTE_INF if best is None else best)
        assert r.tolist() == p


def _random_pieces(rng, K, n_extra=0):
    """K cluster routes over n = sum of sizes stops (sizes 1..4), shuffled."""
    sizes = rng.integers(1, 5, K)
    n = int(sizes.sum()) + n_extra
    perm = rng.permutation(n)[:int(sizes.sum())]
    pieces, at = [], 0
    for s in sizes:
        pieces.append(perm[at:at + s].tolist())
        at += s
    return pieces, n


def test_chain_subsets_match_enumeration():
    """The chaining subset programme (second method) against the plain
    enumeration of every order and orientation, K up to 8 clusters, on
    asymmetric, tie-heavy and INF-bearing matrices."""
    rng = np.random.default_rng(22)
    for case in range(60):
        K = 1 + case % 8
        pieces, n = _random_pieces(rng, K, n_extra=case % 3)
        kind = case % 4
        if kind == 0:
            D = rng.integers(0, 50, (n, n))
        elif kind == 1:
            D = rng.integers(0, 3, (n, n))
        elif kind == 2:
            D = rng.integers(1, 30, (n, n))
            D[rng.random((n, n)) < 0.3] = INF
        else:
            # one stop cut off: every chain infinite while parts stay finite
            D = rng.integers(1, 30, (n, n))
            k = pieces[-1][0]
            D[k, :] = INF
            D[:, k] = INF
        D = D.astype(np.uint32)
        np.fill_diagonal(D, 0)
        c1, r1, cnt = oracle.chain_routes(pieces, D)
        c2, r2, _ = oracle.chain_routes(pieces, D, by_subsets=True)
        assert c1 == c2 and r1.tolist() == r2.tolist(), case
        import math
        assert cnt == math.factorial(K) * 2 ** K


def _py_chain(pieces, D):
    """Cheapest chain by itertools: every order of the pieces times every
    orientation; the smallest (cluster, orientation) sequence among the
    cheapest.  Returns (length or None if infinite, stops)."""
    import itertools
    best = None
    for perm in itertools.permutations(range(len(pieces))):
        for ori in itertools.product((0, 1), repeat=len(pieces)):
            seq = []
            for c, o in zip(perm, ori):
                seq += pieces[c][::-1] if o else pieces[c]
            length = 0
            for a, b in zip(seq, seq[1:]):
                if D[a][b] == INF:
                    length = None
                    break
                length += int(D[a][b])
            key = list(zip(perm, ori))
            if best is None or (length is not None and (best[0] is None or length < best[0])):
                if best is None or length is not None:
                    best = (length, key, seq)
    return best[0], best[2]


def test_clustered_route_by_python_enumeration():
    """Whole clustered routes at 8..12 stops and 4..6 clusters against a
    pure-Python reconstruction: the oracle's K-means partition (pinned on
    its own), each cluster's route by trying every ordering of its stops,
    and the chaining by trying every order and orientation."""
    from oracle.brute import route_by_enumeration
    rng = np.random.default_rng(23)
    for case in range(18):
        n = int(rng.integers(8, 13))
        m = int(rng.integers(4, 7))
        xy = rng.integers(0, 40, (n, 2))
        D = _metric(xy) if case % 2 == 0 else rng.integers(1, 40, (n, n)).astype(np.uint32)
        np.fill_diagonal(D, 0)
        cost, route, mu = oracle.route_clustered(D, xy, m)
        assert mu == m
        asg = oracle.kmeans(xy, m)
        pieces = []
        for c in range(m):
            mem = np.flatnonzero(asg == c)
            if len(mem) == 0:
                continue
            sub = D[np.ix_(mem, mem)].tolist()
            _, r = route_by_enumeration(sub)
            pieces.append(mem[r].tolist())
        length, seq = _py_chain(pieces, D.tolist())
        assert cost == length, (case, cost, length)
        assert route.tolist() == seq, case


def _blob_points(rng, n, m, spread=3, gap=100):
    lab = np.arange(n) % m
    cen = np.array([[gap * c, gap * (c % 2)] for c in range(m)])
    return cen[lab] + rng.integers(-spread, spread + 1, (n, 2)), lab


def test_kmeans_pins():
    from fractions import Fraction
    rng = np.random.default_rng(31)
    # well-separated blobs: the partition is the blobs (up to label order)
    for m in (2, 3, 4):
        xy, lab = _blob_points(rng, 24, m)
        asg = oracle.kmeans(xy, m)
        pairs = {(int(a), int(b)) for a, b in zip(asg, lab)}
        assert len(pairs) == m and len({a for a, _ in pairs}) == m
    # at the end every point sits with its nearest centre (exact rationals),
    # centres being the means of their points: a fixed point of Lloyd's step
    for seed in range(20):
        r = np.random.default_rng(seed)
        n, m = int(r.integers(2, 30)), int(r.integers(1, 6))
        xy = r.integers(0, 40, (n, 2))
        asg = oracle.kmeans(xy, m)
        cents = {}
        for c in set(asg.tolist()):
            pts = xy[asg == c]
            cents[c] = (Fraction(int(pts[:, 0].sum()), len(pts)), Fraction(int(pts[:, 1].sum()), len(pts)))
        for i in range(n):
            d = {c: (xy[i, 0] - cx) ** 2 + (xy[i, 1] - cy) ** 2 for c, (cx, cy) in cents.items()}
            assert d[int(asg[i])] == min(d.values())
    # as many clusters as distinct points: every point is its own cluster
    xy = rng.choice(400, 9, replace=False)
    xy = np.stack([xy % 20, xy // 20], 1)
    assert sorted(oracle.kmeans(xy, 9).tolist()) == list(range(9))


def _metric(xy):
    return np.abs(xy[:, None, :] - xy[None, :, :]).sum(-1).astype(np.uint32)


def test_clustered_route_stitching_by_enumeration():
    """Given the clusters and each cluster's route, the chained route is the
    cheapest of all orderings that keep every cluster's stops together in its
    route's order or the reverse (brute force over all orderings)."""
    import itertools
    rng = np.random.default_rng(32)
    for case in range(16):
        n = int(rng.integers(3, 8))
        m = int(rng.integers(2, 4))
        xy = rng.integers(0, 30, (n, 2))
        D = _metric(xy) if case % 2 == 0 else rng.integers(1, 40, (n, n)).astype(np.uint32)
        np.fill_diagonal(D, 0)
        cost, route, mu = oracle.route_clustered(D, xy, m)
        asg = oracle.kmeans(xy, mu)
        blocks = []
        for c in sorted(set(asg.tolist())):
            mem = np.flatnonzero(asg == c)
            _, r = oracle.route(D[np.ix_(mem, mem)])
            blocks.append(tuple(mem[r].tolist()))
        best = None
        for perm in itertools.permutations(range(n)):
            pos = 0
            ok = True
            seen = set()
            while pos < n:
                b = next((b for b in blocks if perm[pos] in b), None)
                seg = perm[pos:pos + len(b)]
                if b in seen or (seg != b and seg != b[::-1]):
                    ok = False
                    break
                seen.add(b)
                pos += len(b)
            if not ok:
                continue
            length = sum(int(D[a, b]) for a, b in zip(perm, perm[1:]))
            best = length if best is None else min(best, length)
        assert cost == best, (case, cost, best)
        assert sum(int(D[a, b]) for a, b in zip(route, route[1:])) == cost
        assert sorted(route.tolist()) == list(range(n))
        # among the cheapest chains, the smallest (cluster, orientation) sequence
        chains = []
        for perm in itertools.permutations(range(len(blocks))):
            for ori in itertools.product((0, 1), repeat=len(blocks)):
                seq = []
                for c, o in zip(perm, ori):
                    seq += list(blocks[c][::-1] if o else blocks[c])
                length = sum(int(D[a, b]) for a, b in zip(seq, seq[1:]))
                chains.append((length, list(zip(perm, ori)), seq))
        low = min(c[0] for c in chains)
        first = min((c for c in chains if c[0] == low), key=lambda c: c[1])
        assert route.tolist() == first[2], case


def test_clustered_route_limits():
    rng = np.random.default_rng(33)
    for case in range(12):
        n = int(rng.integers(2, 9))
        xy = np.stack([rng.choice(50, n, replace=False), rng.integers(0, 50, n)], 1)
        D = _metric(xy)
        exact, er = oracle.route(D)
        # one cluster: the exact route
        c1, r1, _ = oracle.route_clustered(D, xy, 1)
        assert c1 == exact and r1.tolist() == er.tolist()
        # one stop per cluster: every ordering is a candidate, so exact too
        cn, _, mu = oracle.route_clustered(D, xy, n, max_cluster=20, m_max=8) if n <= 8 else (exact, None, n)
        assert cn == exact
        # any m: never shorter than the exact route
        for m in (2, 3):
            assert oracle.route_clustered(D, xy, m)[0] >= exact
    # a cluster above the size limit raises the cluster count
    xy, _ = _blob_points(rng, 30, 2, spread=4)
    D = _metric(xy)
    _, _, mu = oracle.route_clustered(D, xy, 2, max_cluster=12)
    assert mu > 2
