#!/usr/bin/env python3
"""Benchmark of the warehouse routing hot path on one MI355X.

One step = one wr_order_matrices call over the whole batch of the medium
workload (512x512 rack grid, 256 orders x 32 picks, multi-source relaxation
in one call): planning, relaxation of every distinct pick, and the gather of
all 256 pick-to-pick matrices into device memory.  The graph is uploaded
(and segmented) before the timed region; picks are host index arrays, as the
C ABI defines them.

Prints ONE JSON line:
  value        routed orders/s (whole job; one GPU)
  roofline     dominant kernel (the relaxation pass of the schedule) against HBM:
               algorithmic bytes per launch / its average launch duration,
               timed live with HIP events recorded around each launch
  cpu_baseline the CPU oracle (Dijkstra per distinct pick, all host cores)
               on a bounded sample of the same orders
  route_leg    the next step on the path: exact open routes (wr_order_routes)
               over 12-stop windows of the batch's own matrices, routes/s,
               with its ALU roofline and the CPU oracle beside it; and
               cluster-decomposed routes (wr_order_routes_clustered) over
               the whole 32-pick orders
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
PASS_KERNEL = {"overlay": "k_ovl_pass", "segmented": "k_segb_pass"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--algo", default="overlay")
    ap.add_argument("--tile", type=int, default=512, help="tile vertices (0 = library default)")
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--passes", type=int, default=0)
    ap.add_argument("--segment", default="grid:24x20", help="auto | grid:TWxTH")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU work of the oracle sample (core-seconds)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--b1-orders", type=int, default=2,
                    help="orders of the paper-structured B1 baseline to time (0 = skip)")
    ap.add_argument("--serve-rates", default="500,2000",
                    help="Poisson arrival rates (orders/s) of the serving leg, comma-separated ('' = skip)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window per rate")
    ap.add_argument("--route-stops", type=int, default=12,
                    help="stops per route in the exact-route leg (0 = skip the leg)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device once (a dispatch of known "
                         "traffic that scales the HBM byte counters of a profiler run)")
    return ap.parse_args()


def reach_tables(g):
    """Per-vertex reachable vertex and arc counts.  The workloads have
    symmetric arcs, so the vertices reachable from s form s's connected
    component."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    V = g.V
    rows = np.repeat(np.arange(V), np.diff(g.row_ptr.astype(np.int64)))
    A = sp.csr_matrix((np.ones(g.E, np.int8), (rows, g.col.astype(np.int64))), shape=(V, V))
    ncomp, lab = connected_components(A, directed=True, connection="weak")
    vcount = np.bincount(lab, minlength=ncomp)
    ecount = np.bincount(lab[rows], minlength=ncomp)
    return vcount[lab], ecount[lab]


def kernel_source_sha() -> str:
    p = os.path.join(ROOT, "paper_2504_20655_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch of the pass kernel from the committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", f"{kernel}_medium_traffic.json")))
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


def serving_leg(wr, ctx, rates, seconds, tile):
    """Continuous-batching server on the serving warehouse (3 levels of
    1024x1024 joined by lifts): Poisson order arrivals with sizes uniform in
    2..128, and 1% congestion updates every 100 ms applied between steps.
    Latency is arrival to result ready on the host."""
    from wgen import make_config
    from wgen.orders import CongestionTicker
    wl = make_config("serving")
    g = wl.graph
    ex = wl.extra
    G = wr.Graph(ctx, g.row_ptr, g.col, g.w)
    G.set_schedule(tile, 8, 0)
    G.segment_grid(g.W, g.H, g.levels, 24, 20)
    rng = np.random.default_rng(wl.seed + 7)
    cand = g.aisle_adjacent_vertices()

    def draw(n):
        sizes = rng.integers(ex["pick_lo"], ex["pick_hi"] + 1, n)
        return [cand[rng.choice(len(cand), size=int(P), replace=False)].astype(np.uint32) for P in sizes]

    # warm-up server: builds the tiles, the boundary tables and the captured passes
    srv = wr.Server(G)
    ts = [srv.submit(o) for o in draw(16)]
    srv.drain()
    for t in ts:
        srv.poll(t)
    srv.close()
    out = []
    for rate in rates:
        n = max(1, int(rate * seconds))
        orders = draw(n)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
        ticker = CongestionTicker(np.random.default_rng(wl.seed + 11), g.edge_arc_a, g.edge_arc_b,
                                  g.edge_base_w, g.edge_is_lift, ex["congestion"], ex["congestion_extra"])
        srv = wr.Server(G)
        tickets, ticks = [], 0
        t0 = time.perf_counter()
        next_tick = ex["tick_s"]
        for i in range(n):
            target = t0 + arrivals[i]
            while True:
                now = time.perf_counter()
                if now - t0 >= next_tick:
                    srv.update_weights(*ticker.tick())
                    ticks += 1
                    next_tick += ex["tick_s"]
                if now >= target:
                    break
                time.sleep(min(target - now, 0.0005))
            tickets.append(srv.submit(orders[i]))
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        for t in tickets:
            srv.poll(t)
        srv.close()
        out.append({"rate": rate, "orders": n, "weight_ticks": ticks,
                    "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                    "mean_ms": round(st["mean_ms"], 3), "orders_per_s": round(n / wall, 1),
                    "max_inflight": st["max_inflight_requests"], "steps": st["steps"],
                    "failed": st["failed"]})
        print(f"serving rate {rate}/s: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms "
              f"({n} orders, {ticks} weight ticks)", file=sys.stderr, flush=True)
    G.close()
    return {"workload": "serving: 3 levels of 1024x1024 (V=3,145,728, E=6,422,650), 64 lifts (w=50), "
                        "P ~ U{2..128}, 1% congestion per 100 ms",
            "seconds_per_rate": seconds, "runs": out}


ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 32-bit integer VALU ops: CUs x SIMDs x lanes x clock


def route_leg(wr, ctx, D_host, n_orders, P, stops, steps, warmup, with_cpu):
    """Exact open routes (wr_order_routes) over windows of `stops` picks of
    every order of the batch, cut from the batch's own P x P matrices
    (offsets 0, 4, 8, ... while a window fits): routes/s with the matrices
    resident in HBM, the kernel's ALU roofline (each candidate step of the
    subset programme is an add and a min, n(n-1)2^(n-2) per route), and the
    CPU oracle on a bounded sample."""
    import torch
    mats = [D_host[o * P * P:(o + 1) * P * P].reshape(P, P) for o in range(n_orders)]
    wins = [m[s:s + stops, s:s + stops] for m in mats for s in range(0, P - stops + 1, 4)]
    woff = np.arange(len(wins) + 1, dtype=np.uint32) * stops
    flat = np.concatenate([w.ravel() for w in wins]).astype(np.uint32)
    dev = torch.device("cuda:0")
    d_dist = torch.from_numpy(flat.view(np.int32).copy()).to(dev)
    d_len = torch.zeros(len(wins), dtype=torch.int64, device=dev)
    d_rt = torch.zeros(len(wins) * stops, dtype=torch.int32, device=dev)
    for _ in range(warmup):
        ctx.order_routes(woff, d_dist, d_len, d_rt)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        ctx.order_routes(woff, d_dist, d_len, d_rt)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    n = stops
    ops = 2.0 * n * (n - 1) * 2 ** (n - 2) * len(wins)
    achieved = ops / dt / 1e12
    res = {"workload": f"{len(wins)} routes of {stops} stops: windows of the medium batch's order matrices",
           "value": round(len(wins) / dt, 1), "unit": "routes/s", "ms_per_call": round(dt * 1e3, 4),
           "roofline": {"kernel": "k_route_hk", "bound": "alu", "achieved": round(achieved, 3),
                        "peak": round(ALU_PEAK_TOPS, 1), "unit": "Tops/s",
                        "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": None}}
    # the paper's structure beside it: every ordering in its own thread, on
    # 9-stop windows (9! orderings each), against the subset programme on the
    # same windows
    w9 = [m[s:s + 9, s:s + 9] for m in mats[:16] for s in range(0, P - 9 + 1, 8)]
    o9 = np.arange(len(w9) + 1, dtype=np.uint32) * 9
    f9 = np.concatenate([w.ravel() for w in w9]).astype(np.uint32)
    d9 = torch.from_numpy(f9.view(np.int32).copy()).to(dev)
    l9 = torch.zeros(len(w9), dtype=torch.int64, device=dev)
    r9 = torch.zeros(len(w9) * 9, dtype=torch.int32, device=dev)
    t9 = {}
    for name, en in (("enumerate", True), ("subset_programme", False)):
        ctx.order_routes(o9, d9, l9, r9, enumerate=en)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            ctx.order_routes(o9, d9, l9, r9, enumerate=en)
        torch.cuda.synchronize()
        t9[name] = round(len(w9) * steps / (time.perf_counter() - t), 1)
    res["paper_structure_9_stops"] = {"workload": f"{len(w9)} routes of 9 stops", "unit": "routes/s",
                                      "enumerate_per_thread": t9["enumerate"],
                                      "subset_programme": t9["subset_programme"]}
    if with_cpu:
        import oracle
        k = len(wins)
        t = time.perf_counter()
        oracle.order_routes(woff[:k + 1], flat[:k * stops * stops], nthreads=oracle.max_threads())
        tc = time.perf_counter() - t
        res["cpu_baseline"] = {"value": round(k / tc, 1), "unit": "routes/s", "cores": oracle.max_threads(),
                               "kind": "oracle",
                               "sample": f"first {k} of {len(wins)} routes (Held-Karp in C), {tc:.2f} s wall"}
    return res


def cluster_leg(wr, ctx, D_host, off, picks, W, m, steps, warmup, with_cpu):
    """Cluster-decomposed routes (wr_order_routes_clustered) over every
    order of the batch at full size, positions from the grid: routes/s with
    matrices and positions resident in HBM, and the CPU oracle beside it."""
    import torch
    xy = np.stack([picks % W, picks // W], 1).astype(np.int32)
    n_orders = len(off) - 1
    dev = torch.device("cuda:0")
    d_dist = torch.from_numpy(D_host.view(np.int32).copy()).to(dev)
    d_xy = torch.from_numpy(xy.copy()).to(dev)
    d_len = torch.zeros(n_orders, dtype=torch.int64, device=dev)
    d_rt = torch.zeros(int(off[-1]), dtype=torch.int32, device=dev)
    for _ in range(warmup):
        _, _, used = ctx.order_routes_clustered(off, d_dist, d_xy, m, d_len, d_rt)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        _, _, used = ctx.order_routes_clustered(off, d_dist, d_xy, m, d_len, d_rt)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    res = {"workload": f"{n_orders} orders of {int(off[1] - off[0])} picks, {m} clusters requested "
                       f"(used: {np.bincount(used).tolist()} orders by cluster count)",
           "value": round(n_orders / dt, 1), "unit": "routes/s", "ms_per_call": round(dt * 1e3, 4)}
    if with_cpu:
        import oracle
        t = time.perf_counter()
        oracle.order_routes_clustered(off, D_host, xy, m, m_max=10, nthreads=oracle.max_threads())
        tc = time.perf_counter() - t
        res["cpu_baseline"] = {"value": round(n_orders / tc, 1), "unit": "routes/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"all {n_orders} orders, {tc:.2f} s wall"}
    return res


def cpu_baseline(wl, target_core_s: float):
    import oracle
    g = wl.graph
    off, picks = wl.pick_offsets, wl.picks
    t = time.perf_counter()
    oracle.dijkstra(g.row_ptr, g.col, g.w, int(picks[0]))
    per_src = time.perf_counter() - t
    P = int(off[1] - off[0])
    k = int(max(1, min(wl.num_orders, round(target_core_s / max(per_src, 1e-4) / P))))
    threads = oracle.max_threads()
    sub_off = off[:k + 1]
    sub_picks = picks[:int(sub_off[-1])]
    t = time.perf_counter()
    oracle.order_matrices(g.row_ptr, g.col, g.w, sub_off, sub_picks, nthreads=threads)
    wall = time.perf_counter() - t
    n_src = len(np.unique(sub_picks))
    return {"value": round(k / wall, 3), "unit": "orders/s", "cores": int(min(threads, n_src)),
            "kind": "oracle",
            "sample": f"first {k} of {wl.num_orders} orders ({n_src} distinct picks, one "
                      f"Dijkstra each, {wall:.1f} s wall)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "form of this path is a design note, not a runnable configuration.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2504_20655_amd as wr
    from wgen import make_config

    wl = make_config("medium")
    g = wl.graph
    off, picks = wl.pick_offsets, wl.picks
    n_orders = wl.num_orders
    total = int((np.diff(off.astype(np.int64)) ** 2).sum())

    ctx = wr.Context(0)
    G = wr.Graph(ctx, g.row_ptr, g.col, g.w)
    if args.tile or args.waves or args.passes:
        G.set_schedule(args.tile, args.waves, args.passes)
    if args.segment.startswith("grid:"):
        tw, th = (int(x) for x in args.segment[5:].split("x"))
        G.segment_grid(g.W, g.H, 1, tw, th)
    out = torch.empty(total, dtype=torch.int32, device="cuda")

    # throughput region: passes replayed from captured hipGraphs
    for _ in range(args.warmup):
        G.order_matrices(off, picks, out=out, algo=args.algo)
    torch.cuda.synchronize()
    lat, relax_ms, passes, items = [], 0.0, 0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        G.order_matrices(off, picks, out=out, algo=args.algo)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        info = G.last_run()
        relax_ms += info["relax_ms"]
        passes += info["passes"]
        items += info["work_items"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    info = G.last_run()

    # kernel-timing region: the same steps with HIP events recorded on the
    # library's stream around every launch of the relaxation kernel (passes
    # are launched eagerly so each launch can be bracketed)
    G.order_matrices(off, picks, out=out, algo=args.algo, time_kernels=True)
    kern_ms, kern_n = 0.0, 0
    t1 = time.perf_counter()
    for _ in range(args.steps):
        G.order_matrices(off, picks, out=out, algo=args.algo, time_kernels=True)
        ti = G.last_run()
        kern_ms += ti["kernel_ms"]
        kern_n += ti["kernel_launches"]
    torch.cuda.synchronize()
    eager_ms_step = (time.perf_counter() - t1) / args.steps * 1e3

    # useful work of one step: every distinct pick relaxes its reachable arcs
    vreach, ereach = reach_tables(g)
    uniq = np.unique(picks)
    useful_arcs = float(ereach[uniq].sum())
    # algorithmic HBM bytes: each reached (vertex, source) distance written
    # once and read once (8 B), and each reached arc's (col, w) streamed once
    # per block of 64 sources (8 B / 64)
    alg_bytes = float((8.0 * vreach[uniq] + 8.0 * ereach[uniq] / 64.0).sum())

    ms_per_step = elapsed / args.steps * 1e3
    orders_per_s = n_orders * args.steps / elapsed
    kern_ms_step = kern_ms / args.steps
    launches_step = kern_n / args.steps
    achieved = alg_bytes / (kern_ms_step * 1e-3) / 1e9 if kern_ms_step > 0 else None
    kernel = PASS_KERNEL.get(info["algo"], "relaxation pass")
    traffic = load_traffic(kernel)
    seg = G.segment_info()

    res = {
        "metric": "routed orders/s",
        "value": round(orders_per_s, 1),
        "unit": "orders/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "medium: 512x512 rack-aisle grid (V=262144, E=536188), w in 1..10, "
                        "256 orders x 32 picks, all orders in one multi-source call",
            "orders": n_orders, "picks": int(len(picks)), "unique_sources": int(len(uniq)),
            "algo": info["algo"], "tiles": seg["tiles"], "ports": seg["boundary"],
        },
        "gteps": round(useful_arcs / (ms_per_step * 1e-3) / 1e9, 2),
        "p50_batch_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_batch_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "relax_ms_per_step": round(relax_ms / args.steps, 3),
        "ms_per_step_eager_timed": round(eager_ms_step, 3),
        "passes_per_step": passes / args.steps,
        "visits_per_step": items / args.steps,
        "roofline": {
            "kernel": kernel,
            "bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": (round(traffic * launches_step / (kern_ms_step * 1e-3) / 1e9, 1)
                        if traffic and kern_ms_step > 0 else None),
            "launches_per_step": launches_step,
            "avg_launch_us": round(kern_ms_step / max(launches_step, 1) * 1e3, 2),
            "alg_bytes_per_step": alg_bytes,
        },
    }
    if args.b1_orders > 0:
        k = min(args.b1_orders, n_orders)
        sub_off = off[:k + 1]
        sub_picks = picks[:int(sub_off[-1])]
        sizes = np.diff(sub_off.astype(np.int64))
        o1 = torch.empty(int((sizes ** 2).sum()), dtype=torch.int32, device="cuda")
        t = time.perf_counter()
        G.order_matrices(sub_off, sub_picks, out=o1, algo="edge_b1")
        torch.cuda.synchronize()
        tb = time.perf_counter() - t
        res["baseline_b1"] = {"value": round(k / tb, 3), "unit": "orders/s",
                              "sample": f"first {k} orders, one order at a time, thread per arc, "
                                        f"host-checked early exit ({G.last_run()['passes']} rounds)"}
    if args.route_stops > 0:
        P0 = int(off[1] - off[0])
        if all(int(off[o + 1] - off[o]) == P0 for o in range(n_orders)) and args.route_stops <= P0:
            D_host = out.cpu().numpy().view(np.uint32)[:n_orders * P0 * P0]
            res["route_leg"] = route_leg(wr, ctx, D_host, n_orders, P0, args.route_stops, args.steps,
                                         args.warmup, not args.no_cpu_baseline)
            res["route_leg"]["clustered"] = cluster_leg(wr, ctx, D_host, off, picks, g.W, 3, args.steps,
                                                        args.warmup, not args.no_cpu_baseline)
    rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
    if rates:
        res["serving"] = serving_leg(wr, ctx, rates, args.serve_seconds, args.tile or 512)
    if args.copy_probe > 0:
        n = args.copy_probe << 18
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = int(n) * 4
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
