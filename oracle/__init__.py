"""CPU oracle for the warehouse routing hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it
and shares no code with it.

The C part (``oracle.c`` -> ``liboracle.so``) holds Dijkstra, Jacobi
Bellman-Ford, canonical predecessors, order gathers, CSR validation, the
optimality certificate and the optimal open route over an order's matrix
(Held and Karp's subset programme); ``brute.py`` enumerates simple paths on tiny graphs
and ``closed_forms.py`` holds the grid distance formulas used as pins;
``wms.py`` runs the warehouse reorganisation loop (picking, clustering and
restocking) one run at a time.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

INF = 0xFFFFFFFF
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP over sources)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, os.path.join(_HERE, "oracle.c")])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u32, i32 = ctypes.c_uint32, ctypes.c_int
        L.orc_validate_csr.argtypes = [u32, u32, _u32p, _u32p, _u32p]
        L.orc_validate_csr.restype = i32
        L.orc_dijkstra.argtypes = [u32, _u32p, _u32p, _u32p, u32, _u32p]
        L.orc_dijkstra.restype = i32
        L.orc_dijkstra_multi.argtypes = [u32, _u32p, _u32p, _u32p, u32, _u32p, _u32p, i32]
        L.orc_dijkstra_multi.restype = i32
        L.orc_bellman_ford.argtypes = [u32, _u32p, _u32p, _u32p, u32, _u32p, u32,
                                       ctypes.POINTER(u32)]
        L.orc_bellman_ford.restype = i32
        L.orc_canonical_pred.argtypes = [u32, _u32p, _u32p, _u32p, u32, _u32p, _i32p]
        L.orc_canonical_pred.restype = None
        L.orc_gather_orders.argtypes = [u32, u32, _u32p, _u32p, _u32p, _u32p, _u32p]
        L.orc_gather_orders.restype = None
        L.orc_certificate.argtypes = [u32, _u32p, _u32p, _u32p, u32, _u32p, ctypes.c_void_p]
        L.orc_certificate.restype = i32
        L.orc_certificate_multi.argtypes = [u32, _u32p, _u32p, _u32p, u32, _u32p, _u32p, ctypes.c_void_p,
                                            _i32p, i32]
        L.orc_certificate_multi.restype = i32
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = i32
        _u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
        L.orc_route_held_karp.argtypes = [u32, _u32p, _u64p, _u32p]
        L.orc_route_held_karp.restype = i32
        L.orc_order_routes.argtypes = [u32, _u32p, _u32p, _u64p, _u32p, i32]
        L.orc_order_routes.restype = i32
        L.orc_kmeans.argtypes = [u32, _i32p, u32, _u32p]
        L.orc_kmeans.restype = None
        L.orc_route_clustered.argtypes = [u32, _u32p, _i32p, u32, u32, u32, _u64p, _u32p, _u32p]
        L.orc_route_clustered.restype = i32
        L.orc_order_routes_clustered.argtypes = [u32, _u32p, _u32p, _i32p, u32, u32, u32, _u64p, _u32p, _u32p, i32]
        L.orc_order_routes_clustered.restype = i32
        L.orc_route_enumerate.argtypes = [u32, _u32p, _u64p, _u32p, _u64p]
        L.orc_route_enumerate.restype = i32
        L.orc_chain_routes.argtypes = [u32, _u32p, _u32p, u32, _u32p, i32, _u64p, _u32p, _u64p]
        L.orc_chain_routes.restype = i32
        _lib = L
    return _lib


def _csr(row_ptr, col, w):
    rp = np.ascontiguousarray(row_ptr, dtype=np.uint32)
    c = np.ascontiguousarray(col, dtype=np.uint32)
    ww = np.ascontiguousarray(w, dtype=np.uint32)
    if c.size == 0:   # ndpointer needs a real buffer
        c = np.zeros(1, np.uint32)
        ww = np.zeros(1, np.uint32)
    return rp, c, ww


def validate_csr(row_ptr, col, w) -> int:
    """0 ok, 1 malformed, 2 overflow risk (see oracle.c).  E is the length
    of ``col``; ``w`` must have the same length."""
    E = len(col)
    if len(w) != E:
        return 1
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    if V <= 0:
        return 1
    return lib().orc_validate_csr(V, E, rp, c, ww)


def dijkstra(row_ptr, col, w, src: int) -> np.ndarray:
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    out = np.empty(V, dtype=np.uint32)
    rc = lib().orc_dijkstra(V, rp, c, ww, int(src), out)
    assert rc == 0, rc
    return out


def dijkstra_multi(row_ptr, col, w, sources, nthreads: int = 0) -> np.ndarray:
    """Source-major [S, V] distances, parallel over sources."""
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    src = np.ascontiguousarray(sources, dtype=np.uint32)
    out = np.empty((len(src), V), dtype=np.uint32)
    if len(src):
        rc = lib().orc_dijkstra_multi(V, rp, c, ww, len(src), src, out.reshape(-1), nthreads)
        assert rc == 0, rc
    return out


def bellman_ford(row_ptr, col, w, src: int, max_rounds: int = 0):
    """Jacobi Bellman-Ford; returns (dist, changing_rounds, status)."""
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    out = np.empty(V, dtype=np.uint32)
    r = ctypes.c_uint32(0)
    rc = lib().orc_bellman_ford(V, rp, c, ww, int(src), out, int(max_rounds), ctypes.byref(r))
    return out, int(r.value), rc


def canonical_pred(row_ptr, col, w, src: int, dist) -> np.ndarray:
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    out = np.empty(V, dtype=np.int32)
    lib().orc_canonical_pred(V, rp, c, ww, int(src), d, out)
    return out


def certificate(row_ptr, col, w, src: int, dist, pred=None) -> int:
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    d = np.ascontiguousarray(dist, dtype=np.uint32)
    p = None
    if pred is not None:
        p = np.ascontiguousarray(pred, dtype=np.int32)
    return lib().orc_certificate(V, rp, c, ww, int(src), d,
                                 None if p is None else p.ctypes.data_as(ctypes.c_void_p))


def certificate_rows(row_ptr, col, w, sources, dist, pred=None, nthreads: int = 0) -> np.ndarray:
    """certificate() of every row of a source-major [S, V] distance array
    (and [S, V] predecessors when given), in parallel over sources; returns
    the per-row codes (0 = proven optimal)."""
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    src = np.ascontiguousarray(sources, dtype=np.uint32)
    d = np.ascontiguousarray(dist, dtype=np.uint32).reshape(len(src), V)
    p = None
    if pred is not None:
        p = np.ascontiguousarray(pred, dtype=np.int32).reshape(len(src), V)
    rc = np.zeros(max(len(src), 1), dtype=np.int32)
    if len(src):
        lib().orc_certificate_multi(V, rp, c, ww, len(src), src, d.reshape(-1),
                                    None if p is None else p.ctypes.data_as(ctypes.c_void_p), rc, nthreads)
    return rc[:len(src)]


def order_matrices(row_ptr, col, w, pick_offsets, picks, nthreads: int = 0) -> np.ndarray:
    """Concatenated per-order P x P blocks D_o[i][j] = d(p_i, p_j).

    The distance row of each distinct pick vertex is computed once (it is a
    function of that vertex alone) and read for every (i, j) entry.
    """
    rp, c, ww = _csr(row_ptr, col, w)
    V = len(rp) - 1
    off = np.ascontiguousarray(pick_offsets, dtype=np.uint32)
    pk = np.ascontiguousarray(picks, dtype=np.uint32)
    n_orders = len(off) - 1
    sizes = np.diff(off.astype(np.int64))
    total = int((sizes ** 2).sum())
    out = np.empty(max(total, 1), dtype=np.uint32)
    if total == 0:
        return out[:0]
    uniq, row_of = np.unique(pk, return_inverse=True)
    rows = dijkstra_multi(rp, c, ww, uniq, nthreads)
    lib().orc_gather_orders(V, n_orders, off, pk, row_of.astype(np.uint32),
                            rows.reshape(-1), out)
    return out[:total]


ROUTE_INF = 0xFFFFFFFFFFFFFFFF


def route(D) -> tuple[int, np.ndarray]:
    """Optimal open route over the stops of one n x n matrix (n <= 20):
    (length, lexicographically smallest optimal ordering).  Length is the
    exact sum of the n-1 steps, ROUTE_INF when every ordering meets an INF
    entry.  Held and Karp's programme over stop subsets (C)."""
    M = np.ascontiguousarray(D, dtype=np.uint32)
    n = M.shape[0] if M.ndim == 2 else int(round(len(M) ** 0.5))
    cost = np.zeros(1, dtype=np.uint64)
    r = np.zeros(max(n, 1), dtype=np.uint32)
    if lib().orc_route_held_karp(n, M.reshape(-1) if n else np.zeros(1, np.uint32), cost, r) != 0:
        raise ValueError("route oracle: n out of range or out of memory")
    return int(cost[0]), r[:n]


def order_routes(pick_offsets, dist, nthreads: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """route() of every order: dist holds the concatenated P_o x P_o
    matrices; returns (lengths u64[num_orders], orderings u32[total picks])
    with order o's ordering at pick_offsets[o]."""
    off = np.ascontiguousarray(pick_offsets, dtype=np.uint32)
    n_orders = len(off) - 1
    D = np.ascontiguousarray(dist, dtype=np.uint32)
    cost = np.zeros(max(n_orders, 1), dtype=np.uint64)
    rt = np.zeros(max(int(off[-1]) if n_orders else 0, 1), dtype=np.uint32)
    if n_orders and lib().orc_order_routes(n_orders, off, D if D.size else np.zeros(1, np.uint32),
                                           cost, rt, nthreads) != 0:
        raise ValueError("route oracle: an order is out of range")
    return cost[:n_orders], rt[:int(off[-1]) if n_orders else 0]


def route_enumerate(D) -> tuple[int, np.ndarray, int]:
    """The optimal open route by trying every ordering of the n <= 12 stops
    (C, lexicographic order, first strict improvement kept): (length,
    ordering, orderings compared = n!).  An independent second method
    beside route()."""
    M = np.ascontiguousarray(D, dtype=np.uint32)
    n = M.shape[0]
    cost = np.zeros(1, dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    r = np.zeros(max(n, 1), dtype=np.uint32)
    if lib().orc_route_enumerate(n, M.reshape(-1) if n else np.zeros(1, np.uint32), cost, r, cnt) != 0:
        raise ValueError("route enumeration: n out of range")
    return int(cost[0]), r[:n], int(cnt[0])


def chain_routes(pieces, D, by_subsets: bool = False) -> tuple[int, np.ndarray, int]:
    """Cheapest chaining of cluster routes: pieces is a list of stop-index
    sequences (each a cluster's route over the n x n matrix D); every order
    of the pieces and every orientation of each is a candidate, the chain's
    length adds the pieces' own steps and the steps between consecutive
    pieces.  Returns (length, stops of the chain, chains compared); the
    enumeration compares K! 2^K chains, by_subsets=True uses the subset
    programme instead (count 0)."""
    M = np.ascontiguousarray(D, dtype=np.uint32)
    n = M.shape[0]
    sizes = np.array([len(p) for p in pieces], dtype=np.uint32)
    stops = np.ascontiguousarray(np.concatenate([np.asarray(p) for p in pieces]), dtype=np.uint32)
    cost = np.zeros(1, dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    r = np.zeros(max(len(stops), 1), dtype=np.uint32)
    if lib().orc_chain_routes(len(pieces), sizes, stops, n, M.reshape(-1), 1 if by_subsets else 0,
                              cost, r, cnt) != 0:
        raise ValueError("chain oracle: bad pieces")
    return int(cost[0]), r[:len(stops)], int(cnt[0])


def kmeans(xy, m: int) -> np.ndarray:
    """Cluster of every point (K-means with farthest-point initial centres,
    exact integer comparisons; see orc_route_clustered)."""
    P = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    asg = np.zeros(max(len(P), 1), dtype=np.uint32)
    if len(P):
        lib().orc_kmeans(len(P), P.reshape(-1), m, asg)
    return asg[:len(P)]


def route_clustered(D, xy, m: int, max_cluster: int = 12, m_max: int = 8):
    """Cluster-decomposed route over one order (the Route Optimization
    section's theorem): (length, ordering, clusters used).  The clusters'
    routes are chained by enumerating every order and orientation."""
    M = np.ascontiguousarray(D, dtype=np.uint32)
    n = M.shape[0]
    P = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1)
    cost = np.zeros(1, dtype=np.uint64)
    r = np.zeros(max(n, 1), dtype=np.uint32)
    mu = np.zeros(1, dtype=np.uint32)
    if lib().orc_route_clustered(n, M.reshape(-1) if n else np.zeros(1, np.uint32),
                                 P if n else np.zeros(2, np.int32), m, max_cluster, m_max, cost, r, mu) != 0:
        raise ValueError("clustered route oracle: no cluster count keeps every cluster small")
    return int(cost[0]), r[:n], int(mu[0])


def order_routes_clustered(pick_offsets, dist, xy, m: int, max_cluster: int = 12, m_max: int = 8,
                           nthreads: int = 0):
    """route_clustered() of every order: (lengths u64, orderings u32,
    clusters used u32 per order)."""
    off = np.ascontiguousarray(pick_offsets, dtype=np.uint32)
    n_orders = len(off) - 1
    D = np.ascontiguousarray(dist, dtype=np.uint32)
    P = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1)
    cost = np.zeros(max(n_orders, 1), dtype=np.uint64)
    rt = np.zeros(max(int(off[-1]) if n_orders else 0, 1), dtype=np.uint32)
    mu = np.zeros(max(n_orders, 1), dtype=np.uint32)
    if n_orders and lib().orc_order_routes_clustered(n_orders, off, D if D.size else np.zeros(1, np.uint32),
                                                     P if P.size else np.zeros(2, np.int32), m, max_cluster,
                                                     m_max, cost, rt, mu, nthreads) != 0:
        raise ValueError("clustered route oracle: an order cannot be split into small clusters")
    return cost[:n_orders], rt[:int(off[-1]) if n_orders else 0], mu[:n_orders]


def max_threads() -> int:
    return int(lib().orc_max_threads())
