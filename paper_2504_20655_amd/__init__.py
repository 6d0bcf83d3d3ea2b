"""MI355X warehouse routing: multi-source Bellman-Ford shortest paths, the
segmented (LDS-tile) schedule with boundary exchange, and per-order
pick-to-pick distance matrices, as a C ABI (include/wroute.h) over gfx950
HIP kernels.  This module only marshals arguments for that ABI.

Host arrays are numpy uint32; device outputs may be torch CUDA tensors
(int32 storage holding uint32 bit patterns), in which case the call runs
with WR_DEVICE_PTRS on the tensor's current stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

INF = 0xFFFFFFFF
NO_PRED = -1

DEVICE_PTRS = 0x0001
ALGO = {"auto": 0x00, "sweep": 0x10, "frontier": 0x20, "segmented": 0x30,
        "edge_b1": 0x40, "edge_b0": 0x50, "overlay": 0x60}
ALGO_NAME = {v: k for k, v in ALGO.items()}
NO_GRAPH_CAPTURE = 0x0100
TIME_KERNELS = 0x0200
ROUTE_ENUMERATE = 0x0400
PRUNE_TO_PICKS = 0x0800
DEVICE_INDEX = 0x1000

STATUS = {0: "WR_OK", 1: "WR_E_INVALID", 2: "WR_E_RANGE", 3: "WR_E_NOMEM", 4: "WR_E_DEVICE",
          5: "WR_E_UNSUPPORTED", 6: "WR_E_BUSY", 7: "WR_E_INTERNAL"}
BUSY = 6


class WrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


def lib():
    return _lib.load()


def _check(rc: int):
    if rc != 0:
        raise WrError(rc, (lib().wr_last_error() or b"").decode())


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _is_device(a) -> bool:
    return hasattr(a, "data_ptr") and getattr(a, "is_cuda", False)


def _ptr(a) -> ctypes.c_void_p | None:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(a.ctypes.data or 1)
    return ctypes.c_void_p(a.data_ptr())   # torch tensor


def version() -> str:
    return lib().wr_version().decode()


def debug_fault(kind: str, nth: int = 1):
    """Test hook (wr_debug_fault): the nth next device allocation
    (kind="alloc") or kernel launch (kind="launch") of the library fails on
    the host; kind="off" disarms."""
    _check(lib().wr_debug_fault({"off": 0, "alloc": 1, "launch": 2}[kind], nth))


def validate_csr(row_ptr, col, w) -> int:
    """Returns the wr_status of wr_validate_csr (0 = valid)."""
    rp, c, ww = _u32(row_ptr), _u32(col), _u32(w)
    V = max(len(rp) - 1, 0)
    return lib().wr_validate_csr(V, len(c), _ptr(rp), _ptr(c), _ptr(ww))


class Context:
    def __init__(self, device: int = 0, mem_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(lib().wr_context_create(device, mem_budget_bytes, ctypes.byref(h)))
        self.h = h

    def memory(self):
        used, budget = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().wr_context_memory(self.h, ctypes.byref(used), ctypes.byref(budget)))
        return used.value, budget.value

    def order_routes(self, pick_offsets, dist, lengths=None, routes=None, enumerate: bool = False):
        """Shortest open route over each order's stops (wr_order_routes):
        dist holds the concatenated P x P matrices (numpy uint32, or a device
        tensor with lengths/routes device tensors as well).  enumerate=True
        runs the permutation-per-thread baseline.  Returns (lengths
        uint64[num_orders], orderings uint32[total picks])."""
        off = _u32(pick_offsets)
        n = len(off) - 1
        total = int(off[-1]) if n > 0 else 0
        extra = ROUTE_ENUMERATE if enumerate else 0
        if lengths is not None:
            _check(lib().wr_order_routes(self.h, n, _ptr(off), _ptr(dist), _ptr(lengths), _ptr(routes),
                                         DEVICE_PTRS | extra, _stream_of(lengths)))
            return lengths, routes
        d = _u32(dist)
        ln = np.zeros(max(n, 1), dtype=np.uint64)
        rt = np.zeros(max(total, 1), dtype=np.uint32)
        _check(lib().wr_order_routes(self.h, n, _ptr(off), _ptr(d), _ptr(ln), _ptr(rt), extra, None))
        return ln[:max(n, 0)], rt[:total]

    def order_routes_static(self, pick_offsets, dist, lengths, routes, enumerate: bool = False):
        """wr_order_routes_static: the exact routes of order_routes() with no
        device allocation by the library; dist, lengths (int64) and routes
        (int32) are device tensors, the work runs on lengths' current
        stream.  Returns (lengths, routes)."""
        off = _u32(pick_offsets)
        n = len(off) - 1
        _check(lib().wr_order_routes_static(self.h, n, _ptr(off), _ptr(dist), _ptr(lengths), _ptr(routes),
                                            ROUTE_ENUMERATE if enumerate else 0, _stream_of(lengths)))
        return lengths, routes

    def order_routes_clustered(self, pick_offsets, dist, pick_xy, m: int, lengths=None, routes=None):
        """Cluster-decomposed route over each order's stops
        (wr_order_routes_clustered): pick_xy holds (x, y) per pick.  Returns
        (lengths uint64, orderings uint32, clusters used uint32 per order);
        with device tensors for dist/pick_xy/lengths/routes the call writes
        those in place."""
        off = _u32(pick_offsets)
        n = len(off) - 1
        total = int(off[-1]) if n > 0 else 0
        used = np.zeros(max(n, 1), dtype=np.uint32)
        if lengths is not None:
            _check(lib().wr_order_routes_clustered(self.h, n, _ptr(off), _ptr(dist), _ptr(pick_xy), m,
                                                   _ptr(lengths), _ptr(routes), _ptr(used), DEVICE_PTRS,
                                                   _stream_of(lengths)))
            return lengths, routes, used[:n]
        d = _u32(dist)
        xy = np.ascontiguousarray(pick_xy, dtype=np.int32).reshape(-1)
        ln = np.zeros(max(n, 1), dtype=np.uint64)
        rt = np.zeros(max(total, 1), dtype=np.uint32)
        _check(lib().wr_order_routes_clustered(self.h, n, _ptr(off), _ptr(d), _ptr(xy), m, _ptr(ln), _ptr(rt),
                                               _ptr(used), 0, None))
        return ln[:n], rt[:total], used[:n]

    def wms_run(self, A, M, orders, qty, nx: int, ny: int, nz: int, n_articles: int, mmax: int = 10,
                purchase_orders: int = 20, clusters: int = 3, out=None):
        """The warehouse reorganisation loop (wr_wms_run): `runs`
        independent states A, M [runs, nx*ny*nz] and picking orders
        orders/qty [runs, iters, purchase_orders * articles_per_order]
        (qty may also be [runs, S], the same parcels every iteration).
        Returns (A, M, silhouette [runs, iters], area, moves).  With device
        tensors (A, M, orders, qty int32; out = (silhouette float64, area
        float64, moves int32)) the call runs on the tensors' stream and
        updates A and M in place."""
        if out is not None:
            runs, iters, S = orders.shape
            p = self._wms_params(nx, ny, nz, n_articles, mmax, purchase_orders, S, clusters)
            sil, area, mv = out
            _check(lib().wr_wms_run(self.h, ctypes.byref(p), runs, iters, _ptr(A), _ptr(M), _ptr(orders), _ptr(qty),
                                    _ptr(sil), _ptr(area), _ptr(mv), DEVICE_PTRS, _stream_of(A)))
            return A, M, sil, area, mv
        o = _u32(orders)
        runs, iters, S = o.shape
        q = np.asarray(qty, dtype=np.uint32)
        if q.ndim == 2:
            q = np.broadcast_to(q[:, None, :], o.shape)
        q = np.ascontiguousarray(q)
        a = np.array(A, dtype=np.uint32, order="C", copy=True)
        m = np.array(M, dtype=np.uint32, order="C", copy=True)
        sil = np.zeros((runs, iters))
        area = np.zeros((runs, iters))
        mv = np.zeros((runs, iters), dtype=np.uint32)
        p = self._wms_params(nx, ny, nz, n_articles, mmax, purchase_orders, S, clusters)
        _check(lib().wr_wms_run(self.h, ctypes.byref(p), runs, iters, _ptr(a), _ptr(m), _ptr(o), _ptr(q),
                                _ptr(sil), _ptr(area), _ptr(mv), 0, None))
        return a, m, sil, area, mv

    @staticmethod
    def _wms_params(nx, ny, nz, n_articles, mmax, purchase_orders, S, clusters):
        per = S // purchase_orders if purchase_orders else 0
        if purchase_orders < 1 or per * purchase_orders != S:
            raise ValueError("the order length must be a multiple of purchase_orders")
        return _lib.WmsParams(nx, ny, nz, n_articles, mmax, purchase_orders, per, clusters)

    def close(self):
        if getattr(self, "h", None):
            lib().wr_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_of(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


class Graph:
    """A device-resident CSR graph (wr_graph_create_csr)."""

    def __init__(self, ctx: Context, row_ptr, col, w):
        self.ctx = ctx
        self.row_ptr, self.col, self.w = _u32(row_ptr), _u32(col), _u32(w)
        self.V = len(self.row_ptr) - 1
        self.E = len(self.col)
        h = ctypes.c_void_p()
        _check(lib().wr_graph_create_csr(ctx.h, self.V, self.E, _ptr(self.row_ptr), _ptr(self.col),
                                         _ptr(self.w), 0, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().wr_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # segmentation
    def set_segments(self, segment_of_vertex, num_segments: int):
        s = _u32(segment_of_vertex)
        _check(lib().wr_graph_set_segments(self.h, _ptr(s), int(num_segments)))

    def segment_grid(self, W, H, levels, tile_w, tile_h):
        _check(lib().wr_graph_segment_grid(self.h, W, H, levels, tile_w, tile_h))

    def segment_info(self):
        a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().wr_graph_segment_info(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"segments": a.value, "tiles": b.value, "boundary": c.value}

    def set_schedule(self, tile_vertices=0, waves_per_group=0, passes_per_replay=0):
        _check(lib().wr_graph_set_schedule(self.h, tile_vertices, waves_per_group, passes_per_replay))

    def autotune(self, sources_hint: int = 256, cache_path: str | None = None):
        _check(lib().wr_autotune(self.h, sources_hint, cache_path.encode() if cache_path else None))

    def set_blocks_per_unit(self, blocks: int):
        _check(lib().wr_graph_set_blocks_per_unit(self.h, blocks))

    def schedule(self) -> dict:
        """The schedule the graph runs with (wr_graph_get_schedule)."""
        sc = _lib.Schedule()
        _check(lib().wr_graph_get_schedule(self.h, ctypes.byref(sc)))
        return {k: getattr(sc, k) for k, _ in sc._fields_}

    def update_weights(self, arc_index, new_w) -> int:
        a, v = _u32(arc_index), _u32(new_w)
        ep = ctypes.c_uint64()
        _check(lib().wr_graph_update_weights(self.h, len(a), _ptr(a), _ptr(v), ctypes.byref(ep)))
        return ep.value

    def epoch(self) -> int:
        ep = ctypes.c_uint64()
        _check(lib().wr_graph_epoch(self.h, ctypes.byref(ep)))
        return ep.value

    def last_run(self) -> dict:
        r = _lib.RunInfo()
        _check(lib().wr_graph_last_run(self.h, ctypes.byref(r)))
        d = {k: getattr(r, k) for k, _ in r._fields_}
        d["algo"] = ALGO_NAME.get(d["algo"], d["algo"])
        return d

    # solves
    def sssp(self, sources, pred: bool = False, algo: str = "auto", out=None, pred_out=None,
             graph_capture: bool = True):
        """Distances [S, V] (uint32, source-major); with pred=True also the
        canonical predecessors.  `out`/`pred_out` may be torch CUDA tensors
        of S*V 32-bit elements, in which case results stay on the device."""
        flags = ALGO[algo] | (0 if graph_capture else NO_GRAPH_CAPTURE)
        if _is_device(sources):
            # device sources: read back after the work queued on their stream
            if out is None:
                raise ValueError("device sources need a device `out`")
            S = int(sources.numel())
            _check(lib().wr_sssp(self.h, S, _ptr(sources), _ptr(out), _ptr(pred_out),
                                 flags | DEVICE_PTRS | DEVICE_INDEX, _stream_of(out)))
            return out, pred_out
        src = _u32(sources)
        S = len(src)
        if out is not None:
            flags |= DEVICE_PTRS
            stream = _stream_of(out)
            _check(lib().wr_sssp(self.h, S, _ptr(src), _ptr(out), _ptr(pred_out), flags, stream))
            return out, pred_out
        d = np.empty((S, self.V), dtype=np.uint32)
        p = np.empty((S, self.V), dtype=np.int32) if pred else None
        _check(lib().wr_sssp(self.h, S, _ptr(src), _ptr(d), _ptr(p), flags, None))
        return (d, p) if pred else d

    def order_matrices(self, pick_offsets, picks, pred: bool = False, algo: str = "auto",
                       out=None, pred_out=None, graph_capture: bool = True,
                       time_kernels: bool = False, prune: bool = False):
        """Concatenated per-order P x P matrices (uint32); with pred=True also
        the predecessor row of every pick ([total picks, V]).  prune=True
        sets WR_PRUNE_TO_PICKS.  pick_offsets and picks may be torch CUDA
        tensors (WR_DEVICE_INDEX) when `out` is one too: the call reads them
        after the work queued on the current stream."""
        flags0 = ALGO[algo] | (0 if graph_capture else NO_GRAPH_CAPTURE)
        flags0 |= TIME_KERNELS if time_kernels else 0
        flags0 |= PRUNE_TO_PICKS if prune else 0
        if _is_device(pick_offsets) or _is_device(picks):
            if out is None or not (_is_device(pick_offsets) and _is_device(picks)):
                raise ValueError("device pick_offsets need device picks and a device `out`")
            n = int(pick_offsets.numel()) - 1
            _check(lib().wr_order_matrices(self.h, n, _ptr(pick_offsets), _ptr(picks), _ptr(out),
                                           _ptr(pred_out), flags0 | DEVICE_PTRS | DEVICE_INDEX,
                                           _stream_of(out)))
            return out, pred_out
        off, pk = _u32(pick_offsets), _u32(picks)
        n = len(off) - 1
        sizes = np.diff(off.astype(np.int64))
        total = int((sizes ** 2).sum())
        flags = ALGO[algo] | (0 if graph_capture else NO_GRAPH_CAPTURE)
        flags |= TIME_KERNELS if time_kernels else 0
        flags |= PRUNE_TO_PICKS if prune else 0
        if out is not None:
            flags |= DEVICE_PTRS
            stream = _stream_of(out)
            _check(lib().wr_order_matrices(self.h, n, _ptr(off), _ptr(pk), _ptr(out),
                                           _ptr(pred_out), flags, stream))
            return out, pred_out
        d = np.empty(max(total, 1), dtype=np.uint32)
        p = np.empty((len(pk), self.V), dtype=np.int32) if pred else None
        _check(lib().wr_order_matrices(self.h, n, _ptr(off), _ptr(pk), _ptr(d), _ptr(p), flags, None))
        d = d[:total]
        return (d, p) if pred else d


class Server:
    """Continuous-batching server over a graph (wr_server_*).  The graph must
    stay alive, and must not be used directly, while the server runs."""

    def __init__(self, graph: Graph, max_source_slots: int = 0, mem_budget_bytes: int = 0,
                 max_queue: int = 0, passes_per_step: int = 0, resident_epochs: int = 0):
        from ._lib import ServerOpts
        self.graph = graph
        o = ServerOpts(max_source_slots, mem_budget_bytes, max_queue, passes_per_step, resident_epochs)
        h = ctypes.c_void_p()
        _check(lib().wr_server_create(graph.h, ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._P = {}

    def submit(self, picks) -> int:
        pk = _u32(picks)
        t = ctypes.c_uint64()
        _check(lib().wr_server_submit(self.h, len(pk), _ptr(pk), ctypes.byref(t)))
        self._P[t.value] = len(pk)
        return t.value

    def poll(self, ticket: int):
        """(P x P matrix, info) once done, (None, None) while pending."""
        from ._lib import ReqInfo
        P = self._P[ticket]
        d = np.empty(max(P * P, 1), dtype=np.uint32)
        info = ReqInfo()
        rc = lib().wr_server_poll(self.h, ticket, _ptr(d), ctypes.byref(info))
        if rc == BUSY:
            return None, None
        del self._P[ticket]
        _check(rc)
        return d[:P * P].reshape(P, P), {"epoch": info.epoch, "t_arrive": info.t_arrive,
                                          "t_admit": info.t_admit, "t_done": info.t_done,
                                          "P": info.P, "status": info.status}

    def update_weights(self, arc_index, new_w):
        a, v = _u32(arc_index), _u32(new_w)
        _check(lib().wr_server_update_weights(self.h, len(a), _ptr(a), _ptr(v)))

    def stats(self) -> dict:
        from ._lib import Stats
        s = Stats()
        _check(lib().wr_server_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def drain(self):
        _check(lib().wr_server_drain(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().wr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_matrices(flat, pick_offsets):
    """Splits the concatenated output into a list of P x P arrays."""
    off = np.asarray(pick_offsets, dtype=np.int64)
    res, base = [], 0
    for o in range(len(off) - 1):
        P = int(off[o + 1] - off[o])
        res.append(np.asarray(flat[base:base + P * P]).reshape(P, P))
        base += P * P
    return res
