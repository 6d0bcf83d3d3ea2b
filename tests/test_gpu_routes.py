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
