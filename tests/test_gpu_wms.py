"""GPU parity of the warehouse reorganisation loop (wr_wms_run) against the
oracle (oracle/wms.py), and its error paths.

* 10 x 10 x 10 nodes, 11 empty racks, 20 purchase orders of 10 articles,
  K = 3 (the paper's experiment settings), experiments 1-3, several runs of
  25 iterations: final states and moves bit for bit, silhouettes and areas
  within 1e-14 (both sides take the same correctly rounded square roots and
  divisions in the same order, so they agree exactly in practice).
* 100 x 100 x 10 nodes, 1100 empty racks: a batch of runs as the benchmark
  launches it, sampled runs against the oracle element by element; over the
  batch, the paper's qualitative result (silhouette gains ordered by noise).
* degenerate and edge shapes: no empty node, K = 1, one purchase order,
  more shelves than a 16-bit rack mask holds, K > purchase orders.
* host and device buffers give the same results; bad inputs fail with the
  documented status and leave host buffers unchanged.
"""
import sys

import numpy as np
import pytest

from oracle import wms
from wgen.wms import make_wms

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx(rt):
    return rt.Context(0)


def _run(ctx, s, runs=None, iters=None):
    R = s.A0.shape[0] if runs is None else runs
    T = s.orders.shape[1] if iters is None else iters
    qty = s.qty[:R, :T] if s.qty.ndim == 3 else s.qty[:R]
    return ctx.wms_run(s.A0[:R], s.M0[:R], s.orders[:R, :T], qty, s.nx, s.ny, s.nz, s.n_articles, s.mmax,
                       s.po, s.k)


def _check(s, got, runs, iters=None):
    A, M, sil, area, mv = got
    for r in runs:
        eA, eM, esil, earea, emv = wms.run(s, r, iters)
        assert (A[r] == eA).all(), f"run {r}: states differ at {np.flatnonzero(A[r] != eA)[:5]}"
        assert (M[r] == eM).all(), f"run {r}: balances differ at {np.flatnonzero(M[r] != eM)[:5]}"
        assert (mv[r] == emv).all(), f"run {r}: moves {mv[r][:10]} vs {emv[:10]}"
        assert np.abs(sil[r] - esil).max() <= 1e-14, f"run {r}: silhouette"
        assert np.abs(area[r] - earea).max() <= 1e-14 * max(1.0, np.abs(earea).max()), f"run {r}: area"


@pytest.mark.parametrize("experiment", [1, 2, 3])
def test_paper_warehouse_every_run(ctx, experiment):
    s = make_wms(10 + experiment, 10, 10, 10, 11, 6, 25, experiment)
    got = _run(ctx, s)
    _check(s, got, range(6))
    log(f"exp {experiment}: moves per run {got[4].sum(axis=1).tolist()}")


def test_per_iteration_parcels_and_small_shapes(ctx):
    cases = [make_wms(21, 10, 8, 3, 7, 3, 12, 2, qty_per_iter=True),
             make_wms(22, 6, 5, 20, 3, 2, 10, 3, po=4, per_po=3, k=4),      # 32-bit masks
             make_wms(23, 12, 10, 2, 0, 2, 8, 2),                            # no empty node
             make_wms(24, 9, 7, 4, 5, 2, 8, 3, k=1),                         # one cluster
             make_wms(25, 9, 7, 4, 5, 2, 8, 1, po=1, per_po=40),             # one purchase order
             make_wms(26, 7, 7, 5, 4, 2, 8, 3, po=3, per_po=5, k=6),         # K > purchase orders
             make_wms(27, 40, 3, 16, 6, 2, 8, 2, po=64, per_po=2, mmax=3)]   # 64 points, a full wave
    for s in cases:
        got = _run(ctx, s)
        _check(s, got, range(s.A0.shape[0]))
    A, M, sil, area, mv = _run(ctx, cases[2])
    assert (mv == 0).all()
    A, M, sil, area, mv = _run(ctx, cases[3])
    assert (sil == 0).all() and (area == 0).all()


@pytest.fixture(scope="module")
def large(ctx):
    """The large warehouse of the paper: 100 x 100 x 10 nodes, 1100 empty
    racks, 100 iterations, 16 runs per experiment."""
    res = {}
    for e in (1, 2, 3):
        s = make_wms(30 + e, 100, 100, 10, 1100, 16, 100, e)
        res[e] = (s, _run(ctx, s))
        log(f"large exp {e}: done, moves {res[e][1][4].sum()}")
    return res


@pytest.mark.parametrize("experiment", [1, 2, 3])
def test_large_warehouse_sampled_runs(large, experiment):
    s, got = large[experiment]
    _check(s, got, [0, 11])


def test_large_warehouse_noise_ordering(large):
    """Silhouette gains over 100 iterations fall with the noise level, and
    repeating one order separates the clusters strongly."""
    gain = {}
    for e, (s, got) in large.items():
        sil = got[2]
        gain[e] = float((sil[:, -10:].mean(axis=1) - sil[:, 0]).mean())
    log("large: mean silhouette gains", gain)
    assert gain[1] > gain[2] > gain[3] > 0
    assert gain[1] > 0.5


def test_device_buffers_equal_host(rt, ctx):
    import torch
    s = make_wms(41, 10, 10, 10, 11, 4, 10, 2)
    host = _run(ctx, s)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
    R, T, S = s.orders.shape
    A, M = dev(s.A0), dev(s.M0)
    qty = np.ascontiguousarray(np.broadcast_to(s.qty[:, None, :], (R, T, S)))
    out = (torch.empty((R, T), dtype=torch.float64, device="cuda"),
           torch.empty((R, T), dtype=torch.float64, device="cuda"),
           torch.empty((R, T), dtype=torch.int32, device="cuda"))
    ctx.wms_run(A, M, dev(s.orders), dev(qty), s.nx, s.ny, s.nz, s.n_articles, s.mmax, s.po, s.k, out=out)
    torch.cuda.synchronize()
    assert (A.cpu().numpy().view(np.uint32) == host[0]).all()
    assert (M.cpu().numpy().view(np.uint32) == host[1]).all()
    assert (out[0].cpu().numpy() == host[2]).all() and (out[1].cpu().numpy() == host[3]).all()
    assert (out[2].cpu().numpy().view(np.uint32) == host[4]).all()


def test_bad_inputs(rt, ctx):
    s = make_wms(51, 10, 8, 3, 4, 1, 3, 1)
    base = dict(nx=s.nx, ny=s.ny, nz=s.nz, n_articles=s.n_articles, mmax=s.mmax)

    def call(A=s.A0, M=s.M0, orders=s.orders, qty=s.qty, **kw):
        p = dict(base, **kw)
        return ctx.wms_run(A, M, orders, qty, p["nx"], p["ny"], p["nz"], p["n_articles"], p["mmax"],
                           kw.get("purchase_orders", 20), kw.get("clusters", 3))

    def status(**kw):
        with pytest.raises(rt.WrError) as e:
            call(**kw)
        return e.value.name

    assert status(nz=33) == "WR_E_INVALID"
    assert status(clusters=11) == "WR_E_INVALID"
    assert status(clusters=0) == "WR_E_INVALID"
    assert status(nx=2049) == "WR_E_INVALID"
    A2 = s.A0.copy()
    v = np.flatnonzero(A2[0])[:2]
    A2[0, v[1]] = A2[0, v[0]]                       # one article at two nodes
    assert status(A=A2) == "WR_E_INVALID"
    A3 = s.A0.copy()
    A3[0, v[0]] = s.n_articles + 1                  # an article number above N
    assert status(A=A3) == "WR_E_INVALID"
    o2 = s.orders.copy()
    o2[0, 1, 5] = int(s.A0[0, v[0]])
    A4 = s.A0.copy()
    A4[0, v[0]] = 0                                  # the ordered article is not stored
    assert status(A=A4, orders=o2) == "WR_E_INVALID"
    q2 = s.qty.copy()
    q2[0, 7] = s.mmax + 1
    assert status(qty=q2) == "WR_E_RANGE"
    # the request is unchanged by the failures: the next call is exact
    got = call()
    _check(s, got, [0])


def test_bad_inputs_on_device(rt, ctx):
    """With device buffers the kernel finds the bad state or order and the
    call fails with WR_E_INVALID."""
    import torch
    s = make_wms(52, 10, 8, 3, 4, 1, 3, 1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
    R, T, S = s.orders.shape
    qty = np.ascontiguousarray(np.broadcast_to(s.qty[:, None, :], (R, T, S)))
    out = lambda: (torch.empty((R, T), dtype=torch.float64, device="cuda"),
                   torch.empty((R, T), dtype=torch.float64, device="cuda"),
                   torch.empty((R, T), dtype=torch.int32, device="cuda"))
    A2 = s.A0.copy()
    v = np.flatnonzero(A2[0])[:2]
    A2[0, v[1]] = A2[0, v[0]]
    q2 = qty.copy()
    q2[0, 2, 7] = s.mmax + 1
    for A, q in ((A2, qty), (s.A0, q2)):
        with pytest.raises(rt.WrError) as e:
            ctx.wms_run(dev(A), dev(s.M0), dev(s.orders), dev(q), s.nx, s.ny, s.nz, s.n_articles, s.mmax, s.po,
                        s.k, out=out())
        assert e.value.name == "WR_E_INVALID"
    o = out()
    A, M = dev(s.A0), dev(s.M0)
    ctx.wms_run(A, M, dev(s.orders), dev(qty), s.nx, s.ny, s.nz, s.n_articles, s.mmax, s.po, s.k, out=o)
    torch.cuda.synchronize()
    eA, eM, _, _, emv = wms.run(s, 0)
    assert (A.cpu().numpy().view(np.uint32)[0] == eA).all() and (o[2].cpu().numpy()[0] == emv).all()


@pytest.mark.parametrize("floor", ["paper_10x10x10", "large_100x100x10"])
def test_bench_batches_sampled_runs(rt, ctx, floor):
    """The benchmark's own launches (bench.wms_batch, device buffers, 4,096
    runs on 10x10x10 or 1,792 on 100x100x10, 100 iterations): sampled runs
    against the oracle element by element."""
    import torch
    from bench import wms_batch
    nx, ny, nz, er, runs = (10, 10, 10, 11, 4096) if floor == "paper_10x10x10" else (100, 100, 10, 1100, 1792)
    s = wms_batch(nx, ny, nz, er, runs, 100, 2, 700)
    log(f"{floor}: inputs ready")
    R, T, S = s.orders.shape
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
    A, M = dev(s.A0), dev(s.M0)
    out = (torch.empty((R, T), dtype=torch.float64, device="cuda"),
           torch.empty((R, T), dtype=torch.float64, device="cuda"),
           torch.empty((R, T), dtype=torch.int32, device="cuda"))
    ctx.wms_run(A, M, dev(s.orders), dev(np.broadcast_to(s.qty[:, None, :], (R, T, S))), nx, ny, nz,
                s.n_articles, s.mmax, s.po, s.k, out=out)
    torch.cuda.synchronize()
    sample = [0, R // 2, R - 1]
    A_h = A[sample].cpu().numpy().view(np.uint32)
    M_h = M[sample].cpu().numpy().view(np.uint32)
    sil, area, mv = (out[0][sample].cpu().numpy(), out[1][sample].cpu().numpy(),
                     out[2][sample].cpu().numpy().view(np.uint32))
    del A, M, out
    torch.cuda.empty_cache()
    for q, r in enumerate(sample):
        eA, eM, esil, earea, emv = wms.run(s, r)
        assert (A_h[q] == eA).all() and (M_h[q] == eM).all() and (mv[q] == emv).all(), f"run {r}"
        assert np.abs(sil[q] - esil).max() <= 1e-14 and np.abs(area[q] - earea).max() <= 1e-14 * max(1.0, earea.max())
        log(f"{floor}: run {r} equal to the oracle")
