"""Oracle of the warehouse reorganisation loop -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.  Plain Python over numpy arrays, one run at a time.

The model (Mathematical model section: state space, orders, random
dynamical systems; appendix "WMS loop", Order Processing, Update Stock,
Check Stock and Move Articles, Main): a state x = (A, M) gives the article
type a_v (0 = empty) and the balance m_v of every node v = (i, j, k); an
order o is a list of (article, parcels); filling o from x gives the
intermediate state (A, M - w(x, o)), and a node whose last parcel would be
taken has its article moved to a new location nearer the centre of the
article's cluster, giving x' = f(x, o).  Iterating f over a sequence of
orders is the random dynamical system x_n = f(., o_n) o ... o f(., o_1)(x_0).

Readings where the text is silent (shared with the library; each is listed
in DESIGN):
  W1 clustering: each purchase order (20 of 10 articles in the paper's
     experiments) is the point (sum of i, sum of j) over the rack positions of
     its articles (its size times their mean position); K-means (K = 3 in the
     experiments) as in the clustered-route reading
     (farthest-point start from the first point, Lloyd steps to a fixed
     point, ties to the smaller cluster, exact integer comparisons), run
     before the iteration's picking on the positions at that time;
  W2 a cluster's centre is the mean rack position of its purchase orders'
     articles: S_c / (p n_c) with S_c the sum of its members' points and p
     articles per purchase order;
  W3 picking takes the purchase orders in order and the articles of each in
     order; for article a at node v with q parcels: if m_v > q, m_v -= q;
     else the pick would take the last parcel (m_v <= q): the empty node u
     != v nearest the centre of a's cluster (squared distance of rack
     positions, compared exactly; ties to the smaller node id) takes the
     article if it is strictly nearer than v -- v becomes empty (0, 0) and
     u gets a with mmax - (q - m_v) parcels (restocked full, the remainder
     of the pick taken there) -- otherwise v is restocked in place to
     mmax - (q - m_v);
  W4 metrics of an iteration (on its clustering, before picking): the
     silhouette score of the 20 purchase-order points (Euclidean distance of
     mean positions; s = 0 for a point alone in its cluster or when a = b =
     0) and the area of the triangle of the centres of the first three
     non-empty clusters (0 with fewer than three).
"""
from __future__ import annotations

import math

import numpy as np

from . import kmeans

PO = 20       # purchase orders per picking order in the paper's experiments
PER_PO = 10   # articles per purchase order
K = 3         # clusters


def _rack(v, nx, ny):
    return v % nx, (v // nx) % ny


def cluster_points(pos, order, nx, ny, po=PO):
    """(sum i, sum j) of each purchase order's articles (W1)."""
    per = len(order) // po
    pts = np.zeros((po, 2), np.int64)
    for k in range(po):
        for r in range(per):
            i, j = _rack(int(pos[order[k * per + r]]), nx, ny)
            pts[k, 0] += i
            pts[k, 1] += j
    return pts


def silhouette(pts, asg, per_po=PER_PO):
    """Silhouette score of integer points (scaled by per_po) with labels
    (W4)."""
    n = len(pts)
    d = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            dx, dy = int(pts[i, 0] - pts[j, 0]), int(pts[i, 1] - pts[j, 1])
            d[i, j] = math.sqrt(float(dx * dx + dy * dy)) / float(per_po)
    total = 0.0
    for i in range(n):
        own = [j for j in range(n) if asg[j] == asg[i] and j != i]
        if not own:
            continue
        a = 0.0
        for j in own:
            a += d[i, j]
        a /= len(own)
        b = math.inf
        for c in sorted(set(asg.tolist()) - {int(asg[i])}):
            mem = [j for j in range(n) if asg[j] == c]
            s = 0.0
            for j in mem:
                s += d[i, j]
            b = min(b, s / len(mem))
        if b == math.inf:
            continue
        m = max(a, b)
        total += 0.0 if m == 0.0 else (b - a) / m
    return total / n


def triangle_area(S, cnt, per_po=PER_PO):
    """Area of the triangle of the centres S_c / (p n_c) (W4), from exact
    integers: |cross| / (2 p^2 n_a^2 n_b n_c)."""
    live = [c for c in range(len(cnt)) if cnt[c] > 0]
    if len(live) < 3:
        return 0.0
    a, b, c = live[:3]
    na, nb, nc = int(cnt[a]), int(cnt[b]), int(cnt[c])
    d1x, d1y = int(S[b][0]) * na - int(S[a][0]) * nb, int(S[b][1]) * na - int(S[a][1]) * nb
    d2x, d2y = int(S[c][0]) * na - int(S[a][0]) * nc, int(S[c][1]) * na - int(S[a][1]) * nc
    num = abs(d1x * d2y - d1y * d2x)
    return float(num) / float(2 * per_po * per_po * na * na * nb * nc)


def iterate(A, M, pos, order, qty, nx, ny, mmax, po=PO, k=K):
    """One application of f: clusters, metrics, then picking with moves
    (W1-W4); `order` holds po purchase orders of equal size.  A, M, pos are
    updated in place.  Returns (silhouette, area, moves)."""
    per = len(order) // po
    pts = cluster_points(pos, order, nx, ny, po)
    asg = kmeans(pts, k)
    S = np.zeros((k, 2), np.int64)
    cnt = np.zeros(k, np.int64)
    for p in range(po):
        S[asg[p]] += pts[p]
        cnt[asg[p]] += 1
    sil = silhouette(pts, asg, per)
    area = triangle_area(S, cnt, per)
    moves = 0
    for p in range(po):
        c = int(asg[p])
        scale = per * int(cnt[c])
        sx, sy = int(S[c][0]), int(S[c][1])

        def dist2(v):
            i, j = _rack(v, nx, ny)
            return (scale * i - sx) ** 2 + (scale * j - sy) ** 2

        for r in range(per):
            a = int(order[p * per + r])
            q = int(qty[p * per + r])
            v = int(pos[a])
            m = int(M[v])
            if m > q:
                M[v] = m - q
                continue
            # the empty node nearest the centre, ties to the smaller id
            # (argmin keeps the first of equal values; ids ascend)
            emp = np.flatnonzero(A == 0)
            emp = emp[emp != v]
            best = None
            if len(emp):
                ei, ej = emp % nx, (emp // nx) % ny
                d = (scale * ei - sx) ** 2 + (scale * ej - sy) ** 2
                best = int(emp[int(np.argmin(d))])
            if best is not None and dist2(best) < dist2(v):
                A[v], M[v] = 0, 0
                A[best], M[best] = a, mmax - (q - m)
                pos[a] = best
                moves += 1
            else:
                M[v] = mmax - (q - m)
    return sil, area, moves


def run(setup, r, iters=None):
    """Run r of a WmsSetup (its first `iters` iterations, all by default):
    (final A, final M, silhouette[iters], area[iters], moves[iters])."""
    A = setup.A0[r].astype(np.int64).copy()
    M = setup.M0[r].astype(np.int64).copy()
    pos = np.zeros(setup.n_articles + 1, np.int64)
    for v in np.flatnonzero(A):
        pos[A[v]] = v
    iters = setup.orders.shape[1] if iters is None else iters
    sil = np.zeros(iters)
    area = np.zeros(iters)
    moves = np.zeros(iters, np.int64)
    for it in range(iters):
        qty = setup.qty[r, it] if setup.qty.ndim == 3 else setup.qty[r]
        sil[it], area[it], moves[it] = iterate(A, M, pos, setup.orders[r, it], qty, setup.nx, setup.ny,
                                               setup.mmax, setup.po, setup.k)
    return A.astype(np.uint32), M.astype(np.uint32), sil, area, moves
