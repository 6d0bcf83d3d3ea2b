"""GPU parity of wr_order_routes (shortest open route over each order's
stops, Held and Karp over stop subsets) against the CPU oracle: lengths and
orderings bit-exact, on random matrices that stress the tie-break, INF
steps and asymmetry, and on order matrices the library itself computed."""
import sys

import numpy as np
import pytest

import oracle
from wgen import make_config

pytestmark = pytest.mark.gpu
INF = 0xFFFFFFFF


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx(rt):
    return rt.Context(0)


def _random_mats(rng, sizes):
    mats = []
    for k, n in enumerate(sizes):
        kind = k % 4
        if kind == 0:
            m = rng.integers(0, 1000, (n, n))
        elif kind == 1:
            m = rng.integers(0, 3, (n, n))                       # many ties
        elif kind == 2:
            m = rng.integers(1, 60, (n, n))
            m[rng.random((n, n)) < 0.35] = INF                  # unreachable steps
        else:
            p = rng.integers(0, 50, (n, 2))
            m = np.abs(p[:, None, :] - p[None, :, :]).sum(-1)   # L1 metric
        np.fill_diagonal(m, 0)
        mats.append(m.astype(np.uint32))
    return mats


def _batch(mats):
    off = np.concatenate([[0], np.cumsum([m.shape[0] for m in mats])]).astype(np.uint32)
    flat = np.concatenate([m.ravel() for m in mats]) if mats else np.zeros(0, np.uint32)
    return off, flat.astype(np.uint32)


def test_random_matrices_every_size(rt, ctx):
    rng = np.random.default_rng(21)
    sizes = [n for n in range(0, 13) for _ in range(4)]
    off, flat = _batch(_random_mats(rng, sizes))
    ln, rts = ctx.order_routes(off, flat)
    el, er = oracle.order_routes(off, flat)
    assert np.array_equal(ln, el)
    assert np.array_equal(rts, er)


def test_routes_over_library_matrices(rt, ctx):
    """Orders of up to 12 picks (with a duplicate pick) on a warehouse slice:
    matrices from wr_order_matrices, routes from wr_order_routes."""
    wl = make_config("medium", side=96, num_orders=40)
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.segment_grid(g.W, g.H, 1, 12, 10)
    rng = np.random.default_rng(22)
    sizes = rng.integers(1, 13, 40)
    picks = np.concatenate([rng.choice(wl.picks, s) for s in sizes]).astype(np.uint32)
    picks[1] = picks[0]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    D = G.order_matrices(off, picks, algo="overlay")
    assert np.array_equal(D, oracle.order_matrices(g.row_ptr, g.col, g.w, off, picks))
    ln, rts = ctx.order_routes(off, D)
    el, er = oracle.order_routes(off, D)
    assert np.array_equal(ln, el) and np.array_equal(rts, er)
    # a symmetric metric: a route and its reverse have equal length
    for o in range(len(sizes)):
        r = rts[off[o]:off[o + 1]]
        P = len(r)
        M = D[int((np.diff(off[:o + 1].astype(np.int64)) ** 2).sum()):][:P * P].reshape(P, P)
        fwd = sum(int(M[a, b]) for a, b in zip(r, r[1:]))
        assert fwd == ln[o] == sum(int(M[b, a]) for a, b in zip(r, r[1:]))


def test_device_pointers_match_host(rt, ctx):
    import torch
    rng = np.random.default_rng(23)
    off, flat = _batch(_random_mats(rng, [12, 9, 3, 12, 1, 0, 11]))
    ln, rts = ctx.order_routes(off, flat)
    dev = torch.device("cuda:0")
    d_dist = torch.from_numpy(flat.view(np.int32).copy()).to(dev)
    d_len = torch.zeros(len(off) - 1, dtype=torch.int64, device=dev)
    d_rt = torch.zeros(int(off[-1]), dtype=torch.int32, device=dev)
    ctx.order_routes(off, d_dist, d_len, d_rt)
    torch.cuda.synchronize()
    assert np.array_equal(d_len.cpu().numpy().view(np.uint64), ln)
    assert np.array_equal(d_rt.cpu().numpy().view(np.uint32), rts)


def test_errors(rt, ctx):
    rng = np.random.default_rng(24)
    off, flat = _batch(_random_mats(rng, [13]))
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes(off, flat)
    assert e.value.name == "WR_E_UNSUPPORTED"
    # two finite steps whose sum passes 2^32 - 1
    m = np.array([[0, 3_000_000_000, 3_000_000_000], [3_000_000_000, 0, 3_000_000_000],
                  [3_000_000_000, 3_000_000_000, 0]], np.uint32)
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes(np.array([0, 3], np.uint32), m.ravel())
    assert e.value.name == "WR_E_RANGE"
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes(np.array([0, 3, 2], np.uint32), np.zeros(18, np.uint32))
    assert e.value.name == "WR_E_INVALID"
    ln, rts = ctx.order_routes(np.array([0], np.uint32), np.zeros(0, np.uint32))
    assert len(ln) == 0 and len(rts) == 0


def test_full_batch_twelve_stops(rt, ctx):
    """The benchmark's route workload: 12-pick windows of the medium batch's
    orders (1,536 routes of 12 stops), matrices cut from the batch's own."""
    wl = make_config("medium")
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.set_schedule(512, 8, 0)
    G.segment_grid(g.W, g.H, 1, 24, 20)
    off, picks = wl.pick_offsets, wl.picks
    D = G.order_matrices(off, picks, algo="overlay")
    P = 32
    mats = [D[o * P * P:(o + 1) * P * P].reshape(P, P) for o in range(len(off) - 1)]
    wins = [m[s:s + 12, s:s + 12] for m in mats for s in range(0, 21, 4)]
    woff, wflat = _batch(wins)
    log("routes:", len(wins), "windows of 12 stops")
    ln, rts = ctx.order_routes(woff, wflat)
    rng = np.random.default_rng(25)
    for k in rng.choice(len(wins), 40, replace=False):
        c, r = oracle.route(wins[k])
        assert ln[k] == c and rts[woff[k]:woff[k + 1]].tolist() == r.tolist(), f"window {k}"
    # every length is the length of its own ordering
    for k in range(len(wins)):
        r = rts[woff[k]:woff[k + 1]]
        assert sorted(r.tolist()) == list(range(12))
        assert ln[k] == sum(int(wins[k][a, b]) for a, b in zip(r, r[1:]))


# ------------------------------------------------ cluster-decomposed routes
MMAX = 10   # clusters the library serves (WR_CLUSTER_MAX_CLUSTERS)

def _positions_and_metric(rng, n, span=60):
    xy = rng.integers(0, span, (n, 2)).astype(np.int32)
    D = np.abs(xy[:, None, :] - xy[None, :, :]).sum(-1).astype(np.uint32)
    return xy, D


def test_clustered_random_orders(rt, ctx):
    rng = np.random.default_rng(26)
    sizes = [0, 1, 2, 3, 7, 12, 13, 20, 31, 40, 64, 5, 17, 25, 36, 48]
    mats, xys = [], []
    for k, n in enumerate(sizes):
        xy, D = _positions_and_metric(rng, n)
        if k % 3 == 1:   # an asymmetric matrix over the same positions
            D = (D + rng.integers(0, 7, (n, n))).astype(np.uint32)
            np.fill_diagonal(D, 0)
        if k % 5 == 4:   # some steps cannot be taken (own generator: positions stay as drawn)
            D = D.copy()
            D[np.random.default_rng(100 + k).random((n, n)) < 0.2] = INF
            np.fill_diagonal(D, 0)
        if k == 11:      # no step can be taken: the length is infinite
            D = np.full((n, n), INF, np.uint32)
            np.fill_diagonal(D, 0)
        mats.append(D)
        xys.append(xy)
    off, flat = _batch(mats)
    xy = np.concatenate(xys) if xys else np.zeros((0, 2), np.int32)
    for m in (1, 2, 3, 4, 6, 10):
        ln, rts, used = ctx.order_routes_clustered(off, flat, xy, m)
        el, er, eu = oracle.order_routes_clustered(off, flat, xy, m, m_max=MMAX)
        assert np.array_equal(ln, el), m
        assert np.array_equal(rts, er), m
        assert np.array_equal(used, eu), m
        assert ln[11] == 0xFFFFFFFFFFFFFFFF


def test_clustered_full_batch(rt, ctx):
    """The medium batch's 256 orders of 32 picks, positions from the grid,
    three clusters requested: every order against the oracle, and never
    shorter than the exact route on the orders' 12-pick heads."""
    wl = make_config("medium")
    g = wl.graph
    G = rt.Graph(ctx, g.row_ptr, g.col, g.w)
    G.set_schedule(512, 8, 0)
    G.segment_grid(g.W, g.H, 1, 24, 20)
    off, picks = wl.pick_offsets, wl.picks
    D = G.order_matrices(off, picks, algo="overlay")
    xy = np.stack([picks % g.W, picks // g.W], 1).astype(np.int32)
    ln, rts, used = ctx.order_routes_clustered(off, D, xy, 3)
    log("clustered: clusters used", np.bincount(used).tolist())
    el, er, eu = oracle.order_routes_clustered(off, D, xy, 3, m_max=MMAX)
    assert np.array_equal(ln, el) and np.array_equal(rts, er) and np.array_equal(used, eu)
    P = 32
    heads = [D[o * P * P:(o + 1) * P * P].reshape(P, P)[:12, :12] for o in range(len(off) - 1)]
    hoff, hflat = _batch(heads)
    hxy = np.concatenate([xy[off[o]:off[o] + 12] for o in range(len(off) - 1)])
    exact, _ = ctx.order_routes(hoff, hflat)
    approx, _, _ = ctx.order_routes_clustered(hoff, hflat, hxy, 3)
    assert (approx >= exact).all()
    log("clustered/exact on 12-pick heads: mean", float((approx / exact).mean()))


def test_clustered_device_pointers_and_errors(rt, ctx):
    import torch
    rng = np.random.default_rng(27)
    mats, xys = [], []
    for n in (30, 9, 64, 1):
        xy, D = _positions_and_metric(rng, n)
        mats.append(D)
        xys.append(xy)
    off, flat = _batch(mats)
    xy = np.concatenate(xys)
    ln, rts, used = ctx.order_routes_clustered(off, flat, xy, 3)
    dev = torch.device("cuda:0")
    d_dist = torch.from_numpy(flat.view(np.int32).copy()).to(dev)
    d_xy = torch.from_numpy(xy.copy()).to(dev)
    d_len = torch.zeros(len(off) - 1, dtype=torch.int64, device=dev)
    d_rt = torch.zeros(int(off[-1]), dtype=torch.int32, device=dev)
    _, _, u2 = ctx.order_routes_clustered(off, d_dist, d_xy, 3, d_len, d_rt)
    torch.cuda.synchronize()
    assert np.array_equal(d_len.cpu().numpy().view(np.uint64), ln)
    assert np.array_equal(d_rt.cpu().numpy().view(np.uint32), rts)
    assert np.array_equal(u2, used)
    for m in (0, 11):
        with pytest.raises(rt.WrError) as e:
            ctx.order_routes_clustered(off, flat, xy, m)
        assert e.value.name == "WR_E_INVALID"
    xy65, D65 = _positions_and_metric(rng, 65)
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes_clustered(np.array([0, 65], np.uint32), D65.ravel(), xy65, 3)
    assert e.value.name == "WR_E_UNSUPPORTED"
    bad = xy.copy()
    bad[0, 0] = 1 << 16
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes_clustered(off, flat, bad, 3)
    assert e.value.name == "WR_E_RANGE"
    # forty picks at one position: no number of clusters splits them
    same = np.zeros((40, 2), np.int32)
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes_clustered(np.array([0, 40], np.uint32), np.zeros(1600, np.uint32), same, 2)
    assert e.value.name == "WR_E_UNSUPPORTED"


def test_enumeration_baseline_matches(rt, ctx):
    """The permutation-per-thread baseline (WR_ROUTE_ENUMERATE) returns the
    subset programme's lengths and orderings, and the oracle's, up to 10
    stops; larger orders are refused."""
    rng = np.random.default_rng(28)
    sizes = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 2, 5, 8, 9, 3]
    off, flat = _batch(_random_mats(rng, sizes))
    ln_e, rt_e = ctx.order_routes(off, flat, enumerate=True)
    ln_h, rt_h = ctx.order_routes(off, flat)
    el, er = oracle.order_routes(off, flat)
    assert np.array_equal(ln_e, el) and np.array_equal(rt_e, er)
    assert np.array_equal(ln_h, ln_e) and np.array_equal(rt_h, rt_e)
    off11, flat11 = _batch(_random_mats(rng, [11]))
    with pytest.raises(rt.WrError) as e:
        ctx.order_routes(off11, flat11, enumerate=True)
    assert e.value.name == "WR_E_UNSUPPORTED"
