"""Runs ABI requests through the CPU-executor driver -- TEST INFRASTRUCTURE.

The request format is a flat little-endian uint32 stream read by driver.cpp.
"""
import os
import subprocess
import tempfile

import numpy as np

from tests.simt_cpu.build_cpu import OUT, build

ALGO = {"auto": 0x00, "sweep": 0x10, "frontier": 0x20, "segmented": 0x30,
        "edge_b1": 0x40, "edge_b0": 0x50, "overlay": 0x60, "overlay_prune": 0x60 | 0x800}
NO_GRAPH_CAPTURE = 0x100


def driver(rebuild=False) -> str:
    if rebuild or not os.path.exists(OUT):
        build()
    return OUT


def run(row_ptr, col, w, *, sources=None, pick_offsets=None, picks=None, algo="auto",
        pred=False, graph_capture=True, seg=None, schedule=(0, 0, 0), updates=None, timeout=600,
        server_gap_ms=None, server_updates=(), routes=False, clustered=None):
    """seg: None | ("grid", W, H, L, tw, th) | ("map", nseg, map).  With
    server_gap_ms the orders go through the request server, one every
    server_gap_ms milliseconds, with server_updates = [(arcs, weights,
    orders submitted before it), ...] queued on the way; the matrices are
    then followed by each order's epoch.  With routes=True the order matrices are
    followed by wr_order_routes over them: per order its length (two words,
    low first), then the orderings; clustered=(m, positions) does the same
    with wr_order_routes_clustered and appends the clusters used.  Returns
    (status, out, pred_or_None, stderr)."""
    V = len(row_ptr) - 1
    E = len(col)
    mode = 0 if sources is not None else (2 if server_gap_ms is not None else
                                          (4 if clustered is not None else (3 if routes else 1)))
    flags = server_gap_ms if mode == 2 else ALGO[algo] | (0 if graph_capture else NO_GRAPH_CAPTURE)
    parts = [np.asarray([0x57524F55, mode, flags, 1 if pred else 0, V, E], np.uint32),
             np.asarray(row_ptr, np.uint32), np.asarray(col, np.uint32), np.asarray(w, np.uint32)]
    if seg is None:
        parts.append(np.asarray([0], np.uint32))
    elif seg[0] == "grid":
        parts.append(np.asarray([1, *seg[1:]], np.uint32))
    else:
        parts.append(np.asarray([2, seg[1]], np.uint32))
        parts.append(np.asarray(seg[2], np.uint32))
    parts.append(np.asarray(schedule, np.uint32))
    ua, uv = updates if updates is not None else (np.zeros(0), np.zeros(0))
    parts.append(np.asarray([len(ua)], np.uint32))
    parts.append(np.asarray(ua, np.uint32))
    parts.append(np.asarray(uv, np.uint32))
    if sources is not None:
        src = np.asarray(sources, np.uint32)
        parts += [np.asarray([len(src)], np.uint32), src]
        n_out = len(src) * V
        n_pred = len(src) * V if pred else 0
    else:
        off = np.asarray(pick_offsets, np.uint32)
        pk = np.asarray(picks, np.uint32)
        parts += [np.asarray([len(off) - 1], np.uint32), off, pk]
        if mode == 2:
            parts.append(np.asarray([len(server_updates)], np.uint32))
            for ua_, uw_, after in server_updates:
                parts += [np.asarray([len(ua_)], np.uint32), np.asarray(ua_, np.uint32),
                          np.asarray(uw_, np.uint32), np.asarray([after], np.uint32)]
        if clustered is not None:   # (m, positions int32[2 * picks])
            parts += [np.asarray([clustered[0]], np.uint32), np.asarray(clustered[1], np.int32).view(np.uint32).ravel()]
        sizes = np.diff(off.astype(np.int64))
        n_out = int((sizes ** 2).sum())
        if mode == 2:   # matrices, then each order's epoch
            n_out += len(off) - 1
        if routes:   # matrices, then (length lo, hi) per order, then orderings
            n_out += 2 * (len(off) - 1) + len(pk)
        if clustered is not None:   # ... and the clusters each order used
            n_out += 2 * (len(off) - 1) + len(pk) + (len(off) - 1)
        n_pred = len(pk) * V if pred else 0
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        np.concatenate(parts).astype(np.uint32).tofile(fin)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
        r = subprocess.run([driver(), fin, fout], capture_output=True, text=True, timeout=timeout, env=env)
        if r.returncode != 0 or not os.path.exists(fout):
            raise RuntimeError(f"driver failed rc={r.returncode}\n{r.stderr[-6000:]}")
        res = np.fromfile(fout, dtype=np.uint32)
    status = int(res[0])
    out = res[1:1 + n_out]
    p = res[1 + n_out:1 + n_out + n_pred].view(np.int32) if pred and status == 0 else None
    return status, out, p, r.stderr


def run_wms(setup, runs=None, iters=None, timeout=600):
    """wr_wms_run over a WmsSetup (its first `runs` runs and `iters`
    iterations) through the driver.  Returns (status, A, M, silhouette,
    area, moves, stderr)."""
    R = setup.A0.shape[0] if runs is None else runs
    T = setup.orders.shape[1] if iters is None else iters
    S = setup.orders.shape[2]
    qty = setup.qty[:R, :T] if setup.qty.ndim == 3 else np.broadcast_to(setup.qty[:R, None, :], (R, T, S))
    parts = [np.asarray([0x57524F55, 5, 0, 0, setup.nx, setup.ny, setup.nz, setup.n_articles, setup.mmax,
                         setup.po, S // setup.po, setup.k, R, T], np.uint32),
             setup.A0[:R].ravel(), setup.M0[:R].ravel(), setup.orders[:R, :T].ravel(), np.ascontiguousarray(qty).ravel()]
    V = setup.nx * setup.ny * setup.nz
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        np.concatenate([np.asarray(x, np.uint32).ravel() for x in parts]).tofile(fin)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
        r = subprocess.run([driver(), fin, fout], capture_output=True, text=True, timeout=timeout, env=env)
        if r.returncode != 0 or not os.path.exists(fout):
            raise RuntimeError(f"driver failed rc={r.returncode}\n{r.stderr[-6000:]}")
        res = np.fromfile(fout, dtype=np.uint32)
    status = int(res[0])
    o = 1
    A = res[o:o + R * V].reshape(R, V); o += R * V
    M = res[o:o + R * V].reshape(R, V); o += R * V
    sil = res[o:o + 2 * R * T].view(np.float64).reshape(R, T); o += 2 * R * T
    area = res[o:o + 2 * R * T].view(np.float64).reshape(R, T); o += 2 * R * T
    moves = res[o:o + R * T].reshape(R, T)
    return status, A, M, sil, area, moves, r.stderr
