"""Pins of the warehouse reorganisation oracle (oracle/wms.py) against what
the model and independent routines fix: one iteration worked by hand (moves,
ties, the strictly-nearer rule, restock amounts, the order of picks),
silhouette scores from scikit-learn, triangle areas from a floating-point
formula of their own, the invariants of the state space, and the paper's
qualitative result that repeating one order separates the clusters."""
import numpy as np
import pytest

import oracle
from oracle import wms
from wgen.wms import make_wms


def test_one_iteration_by_hand():
    # a row of six racks (one shelf): articles 1 @ rack 0, 3 @ 1, 4 @ 4,
    # 2 @ 5; racks 2 and 3 empty.  Every purchase order is [1 x5, 2 x5]:
    # all 20 points are (25, 0), one cluster, centre i = 2.5.
    nx, ny, mmax = 6, 1, 10
    A = np.array([1, 3, 0, 0, 4, 2], np.int64)
    M = np.array([10, 10, 0, 0, 10, 10], np.int64)
    pos = np.zeros(5, np.int64)
    for v, a in enumerate(A):
        if a:
            pos[a] = v
    order = np.array(([1] * 5 + [2] * 5) * 20, np.uint32)
    qty = np.ones(200, np.uint32)
    qty[0] = 10   # article 1's first pick would empty rack 0
    qty[5] = 10   # article 2's first pick would empty rack 5
    sil, area, moves = wms.iterate(A, M, pos, order, qty, nx, ny, mmax)
    # article 1: racks 2 and 3 are equally near the centre (0.5) and nearer
    # than rack 0 (2.5): it moves to rack 2 (smaller id), restocked to
    # 10 - (10 - 10) = 10, then 4 picks of 1 -> 6.  Article 2: empty racks 0
    # (2.5) and 3 (0.5), own rack 5 (2.5): moves to rack 3 -> 10, then 6.
    # Purchase orders 1..19 take 95 single parcels of each: 6 -> 1 in 5
    # picks, the 6th finds m = 1 <= q and restocks in place (racks 0 and 5
    # are farther) to 10; 89 more: 8 cycles of 10 leave 10, 9 more leave 1.
    assert A.tolist() == [0, 3, 1, 2, 4, 0]
    assert M.tolist() == [0, 10, 1, 1, 10, 0]
    assert pos[1] == 2 and pos[2] == 3 and moves == 2
    assert sil == 0.0 and area == 0.0   # one cluster: no silhouette, no triangle


@pytest.mark.parametrize("per_po", [10, 3])
def test_silhouette_matches_scikit_learn(per_po):
    from scipy.spatial.distance import cdist
    from sklearn.metrics import silhouette_score
    rng = np.random.default_rng(3 + per_po)
    for case in range(40):
        pts = rng.integers(0, 200, (20, 2))
        if case % 4 == 0:
            pts[5:9] = pts[4]   # coincident points
        labels = rng.integers(0, 3, 20)
        if case % 5 == 0:
            labels[:] = np.arange(20) % 2
        if len(set(labels.tolist())) < 2:
            continue
        # scikit-learn's own Euclidean distances go through |x|^2 + |y|^2 - 2xy
        # and lose ~1e-8; scipy's cdist takes the differences directly
        D = cdist(pts / float(per_po), pts / float(per_po))
        exp = silhouette_score(D, labels, metric="precomputed")
        assert wms.silhouette(pts, labels, per_po) == pytest.approx(exp, rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("per_po", [10, 7])
def test_triangle_area_from_float_centres(per_po):
    rng = np.random.default_rng(4 + per_po)
    for _ in range(200):
        cnt = rng.integers(1, 10, 3)
        S = rng.integers(0, 1000, (3, 2)) * cnt[:, None] + rng.integers(0, 50, (3, 2))
        c = S / (float(per_po) * cnt[:, None])
        (x1, y1), (x2, y2), (x3, y3) = c
        # Heron's formula on the side lengths: a different route to the area
        a, b, d = np.hypot(x2 - x3, y2 - y3), np.hypot(x1 - x3, y1 - y3), np.hypot(x1 - x2, y1 - y2)
        s = (a + b + d) / 2
        heron = np.sqrt(max(s * (s - a) * (s - b) * (s - d), 0.0))
        assert wms.triangle_area(S, cnt, per_po) == pytest.approx(heron, rel=1e-6, abs=1e-6)
        # more clusters: the first three non-empty ones
        S5 = np.vstack([S[:1], np.zeros((1, 2), np.int64), S[1:], rng.integers(0, 9, (1, 2))])
        cnt5 = np.array([cnt[0], 0, cnt[1], cnt[2], 3])
        assert wms.triangle_area(S5, cnt5, per_po) == wms.triangle_area(S, cnt, per_po)
    assert wms.triangle_area(np.ones((3, 2), np.int64), np.array([4, 0, 2])) == 0.0


def test_state_invariants_and_points():
    s = make_wms(11, 10, 8, 3, 5, 1, 25, 3)
    A = s.A0[0].astype(np.int64).copy()
    M = s.M0[0].astype(np.int64).copy()
    pos = np.zeros(s.n_articles + 1, np.int64)
    for v in np.flatnonzero(A):
        pos[A[v]] = v
    empties = int((A == 0).sum())
    for it in range(s.orders.shape[1]):
        order = s.orders[0, it]
        # points from the state by searching A (not through pos)
        pts = wms.cluster_points(pos, order, s.nx, s.ny)
        for k in range(20):
            nodes = [int(np.flatnonzero(A == a)[0]) for a in order[k * 10:(k + 1) * 10]]
            assert pts[k].tolist() == [sum(v % s.nx for v in nodes), sum((v // s.nx) % s.ny for v in nodes)]
        before = M.sum()
        wms.iterate(A, M, pos, order, s.qty[0], s.nx, s.ny, s.mmax)
        # every article once, the empties constant, balances in range, and
        # the balance only moves by the picks plus whole restocks of mmax
        assert sorted(A[A != 0].tolist()) == list(range(1, s.n_articles + 1))
        assert int((A == 0).sum()) == empties
        assert (M >= 0).all() and (M <= s.mmax).all() and (M[A == 0] == 0).all()
        assert all(pos[a] >= 0 and A[pos[a]] == a for a in range(1, s.n_articles + 1))
        picked = int(s.qty[0].astype(np.int64).sum())
        assert (M.sum() - before + picked) % s.mmax == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_repeated_order_separates_clusters(seed):
    """Experiment 1 of the paper (one order over and over on 10x10x10 nodes,
    11 empty racks): the silhouette and the centres' triangle grow; the paper
    reports a silhouette gain of 0.47 on average and areas rising about
    tenfold within 20 iterations."""
    s = make_wms(seed, 10, 10, 10, 11, 1, 60, 1)
    _, _, sil, area, moves = wms.run(s, 0)
    assert sil[-10:].mean() - sil[0] > 0.15
    assert area[-10:].mean() > 2.0 * max(area[0], 0.1)
    assert moves.sum() > 0


def test_small_shape_by_hand():
    """Two purchase orders of two articles, K = 2, on a 4 x 1 floor with two
    shelves: both clusters are single points, so the silhouette is 0 (a point
    alone in its cluster scores 0) and there is no triangle."""
    nx, ny, nz = 4, 1, 2
    # shelf 0: racks 0..3 hold 1, 2, -, 3; shelf 1: 4, -, -, -
    A = np.array([1, 2, 0, 3, 4, 0, 0, 0], np.int64)
    M = np.array([3, 3, 0, 3, 3, 0, 0, 0], np.int64)
    pos = np.zeros(5, np.int64)
    for v in np.flatnonzero(A):
        pos[A[v]] = v
    order = np.array([1, 4, 2, 3], np.uint32)   # PO 0 = {1, 4}: point (0, 0); PO 1 = {2, 3}: (4, 0)
    qty = np.array([3, 1, 2, 3], np.uint32)
    sil, area, moves = wms.iterate(A, M, pos, order, qty, nx, ny, 3, po=2, k=2)
    # PO 0's centre is rack 0 (0/2): article 1 (m = 3 <= 3) looks for the
    # empty node nearest i = 0: nodes 2 (i=2), 5 (i=1), 6 (i=2), 7 (i=3) ->
    # node 5 at distance (2*1 - 0)^2 = 4, not nearer than its own rack 0
    # (0): restocked in place to 3 - (3 - 3) = 3.  Article 4: 3 > 1 -> 2.
    # PO 1's centre is i = 2 (4/2): article 2 at rack 1: 3 > 2 -> 1.
    # Article 3 at rack 3 (3 <= 3): nodes 2 and 6 (rack 2) are both at
    # distance 0 -- ties to node 2 -- strictly nearer than its own (6-4)^2 =
    # 4: it moves to node 2 with 3 - 0 = 3.
    assert A.tolist() == [1, 2, 3, 0, 4, 0, 0, 0]
    assert M.tolist() == [3, 1, 3, 0, 2, 0, 0, 0]
    assert moves == 1 and sil == 0.0 and area == 0.0


def test_kmeans_reading_is_the_route_one():
    # the clustering step is the pinned K-means of the clustered routes
    rng = np.random.default_rng(9)
    pts = rng.integers(0, 100, (20, 2))
    assert (oracle.kmeans(pts, 3) == oracle.kmeans(pts.astype(np.int32), 3)).all()
