#!/usr/bin/env python3
"""Benchmark of the warehouse routing hot path on one MI355X.

Headline (one JSON line): routed orders/s on the uneven-batch workload, the
largest single-GPU order workload: a 2048x2048 rack-aisle grid
(V=4,194,304, E=8,567,292), 10k orders whose pick lists (sizes geometric
with mean 12, clipped to 2..64) are drawn from 100k Zipf(1.1)-popular
slots, all orders in one wr_order_matrices call.  One step = that call with
host pick arrays in and every order's P x P matrix host-visible out:
planning, relaxation of every distinct pick, the gather of all matrices and
their copy to the host.  The graph is uploaded, segmented and autotuned
(grid tile shape, blocks per unit, passes per replay) before the timed
region; the tuning time is reported beside the rate.

Beside the headline:
  roofline      the dominant kernel (the overlay pass) against HBM:
                algorithmic bytes per launch (the byte model: 8 B per
                reached vertex per distinct source + 8 B per reached arc per
                block of 64 sources) / its average launch duration, timed
                live with HIP events on the library's stream; `traffic` is
                the bytes the pass really moves (rocprofv3 FETCH_SIZE and
                WRITE_SIZE, scaled by a copy of known size) per launch over
                the same duration, when the committed counters were taken on
                the current kernel source
  cpu_baseline  the CPU oracle (Dijkstra per distinct pick, all host cores)
                on a bounded sample of the same orders
  legs          medium (512x512, 256 orders x 32 picks), prune (the
                target-bounded variant beside the plain overlay, on uniform
                and window-clustered orders), segmented (4096x4096
                in 256x256 segments, 1024 sources: GTEPS of full distance
                rows, segmented vs unsegmented), tiny (20x40, one order of 8
                picks; the paper-structured baseline in the paper's
                (V-1)E/t convention), the paper-structured baseline B1 (one
                order at a time, thread per arc) on medium and uneven
  route_leg     exact routes over windows of the medium batch's matrices and
                cluster-decomposed routes over its whole orders
  serving       the continuous-batching server on 3 x 1024^2 levels at
                Poisson rates 500, 2000 and 8000 orders/s (p50/p99)
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
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 32-bit integer VALU ops: CUs x SIMDs x lanes x clock
PASS_KERNEL = {"overlay": "k_ovl_pass", "segmented": "k_segb_pass"}
DEFAULT_SEGMENT = (24, 20)   # grid tile the tuner starts from


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--legs", default="medium,segmented,tiny,routes,serving,wms",
                    help="legs beside the uneven headline, comma-separated ('' = none)")
    ap.add_argument("--only", default="", choices=["", "segmented", "tiny", "serving", "wms"],
                    help="run just this leg and print its result (for profiling)")
    ap.add_argument("--no-autotune", action="store_true", help="run the 24x20 grid tiles untuned")
    ap.add_argument("--autotune-cache", default=os.path.join(os.environ.get("TMPDIR", "/tmp"), "wroute_tune"),
                    help="directory of the autotuner's JSON caches")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU work of each oracle sample (core-seconds)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--b1-orders", type=int, default=1,
                    help="orders of the paper-structured B1 baseline to time per workload (0 = skip)")
    ap.add_argument("--serve-rates", default="500,2000,8000",
                    help="Poisson arrival rates (orders/s) of the serving leg, comma-separated")
    ap.add_argument("--serve-seconds", type=float, default=1.5, help="arrival window per rate")
    ap.add_argument("--serve-epochs", default="1,2",
                    help="resident weight epochs of the server to run every rate with, comma-separated")
    ap.add_argument("--route-stops", type=int, default=12, help="stops per route in the exact-route leg")
    ap.add_argument("--wms-runs", default="4096,1792",
                    help="runs per batch of the warehouse-loop leg: 10x10x10 and 100x100x10 warehouses")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device once (a dispatch of known "
                         "traffic that scales the HBM byte counters of a profiler run)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def graph_for(wr, ctx, wl, tune=True, cache_dir=None):
    """The launch configuration the benchmark times (and the full-size
    parity tests check): the workload's grid cut into grid tiles, the
    overlay schedule with tiles of at most 512 vertices, tuned by
    wr_autotune on as many spread sources as the workload has distinct
    picks.  Returns (graph, tuning seconds)."""
    g = wl.graph
    G = wr.Graph(ctx, g.row_ptr, g.col, g.w)
    G.set_schedule(512, 8, 0)
    tw, th = wl.segment_tile or DEFAULT_SEGMENT
    G.segment_grid(g.W, g.H, g.levels, tw, th)
    t = 0.0
    if tune and wl.segment_tile is None:
        hint = int(min(32768, len(np.unique(wl.picks)))) if wl.picks is not None else 4096
        cache = None
        if cache_dir:
            os.makedirs(cache_dir, exist_ok=True)
            cache = os.path.join(cache_dir, f"{wl.name}_{g.W}x{g.H}x{g.levels}.json")
        t0 = time.perf_counter()
        G.autotune(hint, cache)
        t = time.perf_counter() - t0
    return G, t


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


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch of the pass kernel from the committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")))
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


def wms_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("wms.hip", "kmeans_wave.hpp", "wave_ops.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2504_20655_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_wms_instructions():
    """Wave-instructions per run-iteration of k_wms per workload, from the
    committed rocprofv3 counter run, if it was taken on the current source."""
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", "k_wms_instructions.json")))
    except (OSError, ValueError):
        return {}
    if t.get("kernel_src_sha") != wms_source_sha():
        return {}
    return {k: v["wave_instr_per_run_iteration"] for k, v in t.get("workloads", {}).items()}


ISSUE_PEAK = 256 * 4 * 2.4e9   # one wave-instruction per SIMD per cycle


def copy_bandwidth_gbs(mib=2048):
    """Device-to-device copy rate (read + write bytes per second), the
    practical HBM ceiling the measured traffic is also compared with."""
    import torch
    n = mib << 18
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    bw = 2.0 * n * 4 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return bw


def order_leg(wr, wl, G, steps, warmup, tag, host_out=True, copy_gbs=None):
    """Times one whole-batch wr_order_matrices call per step; with host_out
    the matrices come back to host memory inside the timed region."""
    import torch
    g = wl.graph
    off, picks = wl.pick_offsets, wl.picks
    n_orders = wl.num_orders
    total = int((np.diff(off.astype(np.int64)) ** 2).sum())
    out = None if host_out else torch.empty(total, dtype=torch.int32, device="cuda")

    def step():
        if host_out:
            return G.order_matrices(off, picks, algo="overlay")
        G.order_matrices(off, picks, out=out, algo="overlay")
        torch.cuda.synchronize()
        return out

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, passes, items = [], 0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        step()
        lat.append(time.perf_counter() - ts)
        info = G.last_run()
        passes += info["passes"]
        items += info["work_items"]
    elapsed = time.perf_counter() - t0
    log(f"{tag}: {n_orders * steps / elapsed:.0f} orders/s, {elapsed / steps * 1e3:.2f} ms per step")

    # kernel-timing region: the same steps with HIP events recorded on the
    # library's stream around every launch of the pass kernel (passes are
    # launched eagerly so each launch can be bracketed)
    kern_ms, kern_n, kern_bytes, kern_relax = 0.0, 0, 0, 0
    for _ in range(steps):
        G.order_matrices(off, picks, algo="overlay", time_kernels=True)
        ti = G.last_run()
        kern_ms += ti["kernel_ms"]
        kern_n += ti["kernel_launches"]
        kern_bytes += ti["alg_bytes"]
        kern_relax += ti["relaxations"]

    # useful work of one step: every distinct pick relaxes its reachable arcs
    vreach, ereach = reach_tables(g)
    uniq = np.unique(picks)
    useful_arcs = float(ereach[uniq].sum())
    # the plain relaxation's byte model: each reached (vertex, source)
    # distance written and read once, each reached arc streamed once per
    # block of 64 sources; the overlay moves far less than this, so the
    # model's rate is an equivalent bandwidth, not a bound
    model_bytes = float((8.0 * vreach[uniq] + 8.0 * ereach[uniq] / 64.0).sum())
    ms_per_step = elapsed / steps * 1e3
    kern_ms_step = kern_ms / steps
    launches_step = kern_n / steps
    avg_launch_s = kern_ms_step / max(launches_step, 1) * 1e-3
    # the pass's own algorithmic bytes (library counters): a 256-byte row of
    # 64 source values per incoming cross arc and per exit of every visited
    # tile, 4 bytes per exit value stored
    alg_per_launch = kern_bytes / max(kern_n, 1)
    achieved = alg_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else None
    model_gbs = model_bytes / max(launches_step, 1) / avg_launch_s / 1e9 if avg_launch_s > 0 else None
    traffic_b = load_traffic("k_ovl_pass", wl.name)
    traffic = traffic_b / avg_launch_s / 1e9 if traffic_b and avg_launch_s > 0 else None
    seg = G.segment_info()
    res = {
        "orders_per_s": round(n_orders * steps / elapsed, 1),
        "ms_per_step": round(ms_per_step, 4),
        "p50_batch_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_batch_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "output": "host" if host_out else "device",
        "orders": n_orders, "picks": int(len(picks)), "unique_sources": int(len(uniq)),
        "matrix_entries": total,
        "gteps": round(useful_arcs / (ms_per_step * 1e-3) / 1e9, 2),
        "passes_per_step": passes / steps,
        "visits_per_step": items / steps,
        "schedule": G.schedule(), "tiles": seg["tiles"], "ports": seg["boundary"],
        "roofline": {
            "kernel": "k_ovl_pass", "bound": "hbm",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": round(traffic, 1) if traffic else None,
            "traffic_frac": round(traffic / HBM_PEAK_GBS, 4) if traffic else None,
            "traffic_vs_copy": round(traffic / copy_gbs, 4) if traffic and copy_gbs else None,
            "traffic_bytes_per_launch": traffic_b,
            "alg_bytes_per_launch": round(alg_per_launch),
            "launches_per_step": launches_step,
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "kernel_ms_per_step": round(kern_ms_step, 3),
            "plain_bf_model_gbs": round(model_gbs, 1) if model_gbs else None,
            "plain_bf_model_bytes_per_step": model_bytes,
        },
        "relaxations_per_s": round(kern_relax / max(kern_ms, 1e-9) * 1e3, 1),
    }
    return res


def prune_leg(wr, G, wl, steps, warmup):
    """The target-bounded variant (WR_PRUNE_TO_PICKS) beside the plain
    overlay on the medium graph: the medium batch (uniform picks) and a batch
    of 256 orders whose 32 picks lie in a 48x48-cell window each (as after
    the paper's reorganisation has gathered an order's articles)."""
    from wgen.orders import window_orders
    g = wl.graph
    rng = np.random.default_rng(wl.seed + 31)
    coff, cpicks = window_orders(rng, g.aisle_adjacent_vertices(), g.W, g.H, 256, 32, 48)
    out = {}
    for name, off, picks in (("uniform", wl.pick_offsets, wl.picks), ("clustered", coff, cpicks)):
        row = {}
        for tag, pr in (("overlay", False), ("pruned", True)):
            for _ in range(warmup):
                G.order_matrices(off, picks, algo="overlay", prune=pr)
            t = time.perf_counter()
            for _ in range(steps):
                G.order_matrices(off, picks, algo="overlay", prune=pr)
            dt = (time.perf_counter() - t) / steps
            info = G.last_run()
            row[tag] = {"orders_per_s": round((len(off) - 1) / dt, 1), "ms_per_step": round(dt * 1e3, 3),
                        "passes": info["passes"], "visits": info["work_items"]}
        out[name] = row
    return {"workload": "medium graph; uniform: the medium batch; clustered: 256 orders x 32 picks, each in a "
                        "48x48-cell window; matrices copied to the host", **out}


def cpu_orders_baseline(wl, core_seconds):
    """The oracle (one Dijkstra per distinct pick, all host threads) on the
    first orders of the batch, sized to about `core_seconds` of CPU work."""
    import oracle
    g = wl.graph
    off, picks = wl.pick_offsets, wl.picks
    t = time.perf_counter()
    oracle.dijkstra(g.row_ptr, g.col, g.w, int(picks[0]))
    per_src = time.perf_counter() - t
    mean_p = len(picks) / max(wl.num_orders, 1)
    k = int(max(1, min(wl.num_orders, round(core_seconds / max(per_src, 1e-4) / mean_p))))
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


def b1_leg(G, wl, k):
    """The paper's structure on the same GPU: one order at a time, one
    thread per arc, the order's picks looped in each thread, one launch per
    round and a host-read changed flag."""
    import torch
    off, picks = wl.pick_offsets, wl.picks
    k = min(k, wl.num_orders)
    sub_off = off[:k + 1]
    sub_picks = picks[:int(sub_off[-1])]
    sizes = np.diff(sub_off.astype(np.int64))
    o1 = torch.empty(int((sizes ** 2).sum()), dtype=torch.int32, device="cuda")
    t = time.perf_counter()
    G.order_matrices(sub_off, sub_picks, out=o1, algo="edge_b1")
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    return {"value": round(k / tb, 3), "unit": "orders/s",
            "sample": f"first {k} orders, one order at a time, thread per arc, "
                      f"host-checked early exit ({G.last_run()['passes']} rounds)"}


def segmented_leg(wr, ctx, steps):
    """4096x4096 grid in 256x256-cell segments (cut into LDS tiles of at most
    512 vertices), 1024 sources: full distance rows of every source into
    device memory (GTEPS), the 1024 x 1024 matrix between the sources, and
    the unsegmented frontier schedule on a bounded sample of sources."""
    import torch
    from wgen import make_config
    wl = make_config("segmented")
    g = wl.graph
    src = wl.sources
    G, _ = graph_for(wr, ctx, wl, tune=False)
    vreach, ereach = reach_tables(g)
    useful = float(ereach[src].sum())
    out = torch.empty(len(src) * g.V, dtype=torch.int32, device="cuda")
    G.sssp(src, algo="overlay", out=out)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = max(1, min(steps, 3))
    for _ in range(reps):
        G.sssp(src, algo="overlay", out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    info = G.last_run()
    log(f"segmented: {info}")
    del out
    torch.cuda.empty_cache()
    log(f"segmented: {len(src)} full rows in {dt * 1e3:.1f} ms")
    off = np.array([0, len(src)], dtype=np.uint32)
    mo = torch.empty(len(src) ** 2, dtype=torch.int32, device="cuda")
    G.order_matrices(off, src, out=mo, algo="overlay")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        G.order_matrices(off, src, out=mo, algo="overlay")
    torch.cuda.synchronize()
    dm = (time.perf_counter() - t) / reps
    # unsegmented: the frontier schedule over the whole graph, one source
    # at a time (its cost per source grows with the sources sharing a block)
    ns = 2
    fo = torch.empty(g.V, dtype=torch.int32, device="cuda")
    t = time.perf_counter()
    for i in range(ns):
        G.sssp(src[i:i + 1], algo="frontier", out=fo)
    torch.cuda.synchronize()
    df = (time.perf_counter() - t) / ns
    seg = G.segment_info()
    G.close()
    return {"workload": f"segmented: 4096x4096 rack-aisle grid (V={g.V}, E={g.E}), 256x256-cell segments "
                        f"({seg['tiles']} LDS tiles, {seg['boundary']} ports), {len(src)} sources",
            "full_rows_ms": round(dt * 1e3, 3), "gteps": round(useful / dt / 1e9, 2),
            "relax_ms": round(info["relax_ms"], 3),
            "passes": info["passes"], "visits": info["work_items"],
            "matrix_1024_ms": round(dm * 1e3, 3),
            "segmented_ms_per_source": round(dt * 1e3 / len(src), 4),
            "unsegmented_frontier_ms_per_source": round(df * 1e3, 3),
            "unsegmented_sample": f"{ns} sources, one per call, frontier schedule",
            "segmented_speedup_per_source": round(df / (dt / len(src)), 1)}


def tiny_leg(wr, ctx, steps):
    """20x40 grid, one order of 8 picks: the overlay call (µs per order) and
    the paper-faithful baseline B0 (exactly V-1 rounds, the 8 picks looped in
    each arc's thread), quoted in the paper's (V-1)E/t convention."""
    import torch
    from wgen import make_config
    wl = make_config("tiny")
    g = wl.graph
    G, _ = graph_for(wr, ctx, wl, tune=False)
    off, picks = wl.pick_offsets, wl.picks
    out = torch.empty(64, dtype=torch.int32, device="cuda")
    G.order_matrices(off, picks, out=out, algo="overlay")
    torch.cuda.synchronize()
    n = max(steps, 20)
    t = time.perf_counter()
    for _ in range(n):
        G.order_matrices(off, picks, out=out, algo="overlay")
    torch.cuda.synchronize()
    do = (time.perf_counter() - t) / n
    rows = torch.empty(len(picks) * g.V, dtype=torch.int32, device="cuda")
    G.sssp(picks, algo="edge_b0", out=rows)
    torch.cuda.synchronize()
    t = time.perf_counter()
    G.sssp(picks, algo="edge_b0", out=rows)
    torch.cuda.synchronize()
    d0 = time.perf_counter() - t
    r0 = G.last_run()["passes"]
    t = time.perf_counter()
    G.sssp(picks, algo="edge_b1", out=rows)
    torch.cuda.synchronize()
    d1 = time.perf_counter() - t
    r1 = G.last_run()["passes"]
    G.close()
    return {"workload": f"tiny: 20x40 grid (V={g.V}, E={g.E}), 1 order x 8 picks",
            "overlay_us_per_order": round(do * 1e6, 1),
            "b0_ms": round(d0 * 1e3, 3), "b0_rounds": r0,
            "b0_mteps_paper_convention": round((g.V - 1) * g.E / d0 / 1e6, 1),
            "b1_ms": round(d1 * 1e3, 3), "b1_rounds": r1,
            "paper_context": "2627 MTEPS at V=9,716, E=26,999 on an RTX 6000 (GPU Implementation subsection)"}


def serving_leg(wr, ctx, rates, seconds, epochs=(1,)):
    """Continuous-batching server on the serving warehouse (3 levels of
    1024x1024 joined by lifts): Poisson order arrivals with sizes uniform in
    2..128, and 1% congestion updates every 100 ms applied between steps.
    Latency is arrival to result ready on the host."""
    from wgen import make_config
    from wgen.orders import CongestionTicker
    wl = make_config("serving")
    g = wl.graph
    ex = wl.extra
    G, _ = graph_for(wr, ctx, wl, tune=False)
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
    for rate, ep in ((r, e) for e in epochs for r in rates):
        n = max(1, int(rate * seconds))
        orders = draw(n)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
        ticker = CongestionTicker(np.random.default_rng(wl.seed + 11), g.edge_arc_a, g.edge_arc_b,
                                  g.edge_base_w, g.edge_is_lift, ex["congestion"], ex["congestion_extra"])
        srv = wr.Server(G, resident_epochs=ep)
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
        t_sub = time.perf_counter() - t0
        srv.drain()
        wall = time.perf_counter() - t0
        st = srv.stats()
        for t in tickets:
            srv.poll(t)
        srv.close()
        out.append({"rate": rate, "resident_epochs": ep, "orders": n, "weight_ticks": ticks,
                    "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                    "mean_ms": round(st["mean_ms"], 3), "orders_per_s": round(n / wall, 1),
                    "arrival_window_s": round(t_sub, 3), "wall_s": round(wall, 3),
                    "saturated": bool(n / wall < 0.9 * rate),
                    "max_inflight": st["max_inflight_requests"], "steps": st["steps"],
                    "failed": st["failed"]})
        log(f"serving rate {rate}/s, {ep} resident epoch(s): {n / wall:.0f} orders/s completed, p50 {st['p50_ms']:.2f} ms "
            f"p99 {st['p99_ms']:.2f} ms ({n} orders, {ticks} weight ticks)")
    G.close()
    return {"workload": "serving: 3 levels of 1024x1024 (V=3,145,728, E=6,422,650), 64 lifts (w=50), "
                        "P ~ U{2..128}, 1% congestion per 100 ms",
            "seconds_per_rate": seconds, "runs": out}


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


def wms_batch(nx, ny, nz, empty_racks, runs, iters, experiment, seed):
    """Seeded states and orders of `runs` independent runs, generated in
    groups of 64 runs (the generator's loops are per run)."""
    from wgen.wms import make_wms
    parts = [make_wms(seed + g, nx, ny, nz, empty_racks, min(64, runs - g), iters, experiment)
             for g in range(0, runs, 64)]
    s = parts[0]
    s.A0 = np.concatenate([p.A0 for p in parts])
    s.M0 = np.concatenate([p.M0 for p in parts])
    s.orders = np.concatenate([p.orders for p in parts])
    s.qty = np.concatenate([p.qty for p in parts])
    return s


def wms_leg(wr, ctx, runs_small, runs_large, steps, warmup, with_cpu, cpu_seconds):
    """The warehouse reorganisation loop (wr_wms_run), experiment 2 (one
    random article per purchase order), 100 iterations per run and step,
    on the paper's 10x10x10 warehouse (11 empty racks) and its 100x100x10
    one (1100 empty racks): run-iterations/s (applications of f) with the
    states and orders resident in HBM, each step continuing the runs from
    the previous step's states; the oracle beside it on one run."""
    import torch
    from oracle import wms as owms
    dev = torch.device("cuda:0")
    instr = load_wms_instructions()
    out = {}
    for name, (nx, ny, nz, er, runs) in (("paper_10x10x10", (10, 10, 10, 11, runs_small)),
                                         ("large_100x100x10", (100, 100, 10, 1100, runs_large))):
        if runs <= 0:
            continue
        iters = 100
        s = wms_batch(nx, ny, nz, er, runs, iters, 2, 700)
        R, T, S = s.orders.shape
        tens = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)
        A, M = tens(s.A0), tens(s.M0)
        d_ord = tens(s.orders)
        d_qty = tens(np.broadcast_to(s.qty[:, None, :], (R, T, S)))
        res = (torch.empty((R, T), dtype=torch.float64, device=dev),
               torch.empty((R, T), dtype=torch.float64, device=dev),
               torch.empty((R, T), dtype=torch.int32, device=dev))
        call = lambda: ctx.wms_run(A, M, d_ord, d_qty, nx, ny, nz, s.n_articles, s.mmax, s.po, s.k, out=res)
        for _ in range(warmup):
            call()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        leg = {"workload": f"{nx}x{ny}x{nz} nodes, {er} empty racks, {R} runs x {T} iterations of "
                           f"20 purchase orders x 10 articles, K=3, experiment 2",
               "value": round(R * T / dt, 1), "unit": "run-iterations/s", "ms_per_step": round(dt * 1e3, 3),
               "moves_per_iteration": round(float(res[2].double().mean()), 2),
               "silhouette_last": round(float(res[0][:, -1].mean()), 4)}
        # a dependent chain per run: the bound is instruction issue; the
        # instructions per run-iteration come from the profiler's counters
        per = instr.get(name)
        leg["roofline"] = {"kernel": "k_wms", "bound": "issue", "unit": "T wave-instructions/s",
                           "peak": round(ISSUE_PEAK / 1e12, 3), "traffic": None,
                           "achieved": round(per * R * T / dt / 1e12, 4) if per else None,
                           "frac": round(per * R * T / dt / ISSUE_PEAK, 4) if per else None,
                           "wave_instr_per_run_iteration": per}
        if with_cpu:
            # the oracle on run 0 from the initial state, as many iterations
            # as fit the CPU budget
            t = time.perf_counter()
            k = 0
            A0 = s.A0[0].astype(np.int64).copy()
            M0 = s.M0[0].astype(np.int64).copy()
            pos = np.zeros(s.n_articles + 1, np.int64)
            for v in np.flatnonzero(A0):
                pos[A0[v]] = v
            while k < T and time.perf_counter() - t < cpu_seconds / 2:
                owms.iterate(A0, M0, pos, s.orders[0, k], s.qty[0], nx, ny, s.mmax, s.po, s.k)
                k += 1
            tc = time.perf_counter() - t
            leg["cpu_baseline"] = {"value": round(k / tc, 2), "unit": "run-iterations/s", "cores": 1,
                                   "kind": "oracle", "sample": f"run 0, first {k} iterations, {tc:.2f} s"}
        out[name] = leg
        del A, M, d_ord, d_qty, res
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the multi-GPU "
              "form of this path is a design note, not a runnable configuration.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2504_20655_amd as wr
    from wgen import make_config

    legs = [x.strip() for x in args.legs.split(",") if x.strip()]
    with_cpu = not args.no_cpu_baseline
    ctx = wr.Context(0)
    if args.only:
        if args.only == "segmented":
            leg = segmented_leg(wr, ctx, args.steps)
        elif args.only == "tiny":
            leg = tiny_leg(wr, ctx, args.steps)
        elif args.only == "wms":
            rs = [int(x) for x in args.wms_runs.split(",")]
            leg = wms_leg(wr, ctx, rs[0], rs[1], args.steps, args.warmup, not args.no_cpu_baseline,
                          args.cpu_seconds)
        else:
            leg = serving_leg(wr, ctx, [float(x) for x in args.serve_rates.split(",") if x.strip()],
                              args.serve_seconds, [int(x) for x in args.serve_epochs.split(",") if x.strip()])
        print(json.dumps({"leg": args.only, **leg}), flush=True)
        return
    copy_gbs = copy_bandwidth_gbs()

    # headline: the uneven batch, matrices host-visible
    wl = make_config("uneven")
    log(f"uneven: {wl.num_orders} orders, {len(wl.picks)} picks")
    G, tune_s = graph_for(wr, ctx, wl, tune=not args.no_autotune, cache_dir=args.autotune_cache)
    log(f"uneven: tuned in {tune_s:.1f} s: {G.schedule()}")
    head = order_leg(wr, wl, G, args.steps, args.warmup, "uneven", host_out=True, copy_gbs=copy_gbs)
    head["autotune_s"] = round(tune_s, 2)
    if args.b1_orders > 0:
        head["baseline_b1"] = b1_leg(G, wl, args.b1_orders)
    G.close()
    roof = head.pop("roofline")
    res = {
        "metric": "routed orders/s",
        "value": head["orders_per_s"],
        "unit": "orders/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "uneven: 2048x2048 rack-aisle grid (V=4194304, E=8567292), w in 1..10, 10k orders "
                        "with geometric(12) sizes in 2..64 over 100k Zipf(1.1) slots, all orders in one "
                        "autotuned multi-source call, matrices host-visible",
            "orders": head["orders"], "picks": head["picks"], "unique_sources": head["unique_sources"],
            "algo": "overlay", "schedule": head["schedule"], "tiles": head["tiles"], "ports": head["ports"],
        },
        "gteps": head["gteps"],
        "p50_batch_ms": head["p50_batch_ms"],
        "p99_batch_ms": head["p99_batch_ms"],
        "passes_per_step": head["passes_per_step"],
        "visits_per_step": head["visits_per_step"],
        "autotune_s": head["autotune_s"],
        "relaxations_per_s": head["relaxations_per_s"],
        "copy_gbs": round(copy_gbs, 1),
        "roofline": roof,
    }
    if "baseline_b1" in head:
        res["baseline_b1"] = head["baseline_b1"]
    if with_cpu:
        res["cpu_baseline"] = cpu_orders_baseline(wl, args.cpu_seconds)
    res["legs"] = {}
    del wl

    if "medium" in legs or "routes" in legs:
        wm = make_config("medium")
        Gm, tm = graph_for(wr, ctx, wm, tune=not args.no_autotune, cache_dir=args.autotune_cache)
        med = order_leg(wr, wm, Gm, args.steps * 2, args.warmup, "medium", host_out=True, copy_gbs=copy_gbs)
        dev_leg = order_leg(wr, wm, Gm, args.steps * 2, args.warmup, "medium (device)", host_out=False,
                            copy_gbs=copy_gbs)
        med["device_output"] = {k: dev_leg[k] for k in ("orders_per_s", "ms_per_step", "p50_batch_ms",
                                                          "p99_batch_ms", "gteps")}
        med["autotune_s"] = round(tm, 2)
        if args.b1_orders > 0:
            med["baseline_b1"] = b1_leg(Gm, wm, 2 * args.b1_orders)
        if with_cpu:
            med["cpu_baseline"] = cpu_orders_baseline(wm, args.cpu_seconds)
        res["legs"]["medium"] = med
        res["legs"]["prune"] = prune_leg(wr, Gm, wm, args.steps, args.warmup)
        if "routes" in legs and args.route_stops > 0:
            off, picks = wm.pick_offsets, wm.picks
            P0 = int(off[1] - off[0])
            D_host = Gm.order_matrices(off, picks, algo="overlay")
            res["route_leg"] = route_leg(wr, ctx, D_host, wm.num_orders, P0, args.route_stops, args.steps,
                                         args.warmup, with_cpu)
            res["route_leg"]["clustered"] = cluster_leg(wr, ctx, D_host, off, picks, wm.graph.W, 3, args.steps,
                                                        args.warmup, with_cpu)
        Gm.close()
        torch.cuda.empty_cache()
    if "tiny" in legs:
        res["legs"]["tiny"] = tiny_leg(wr, ctx, args.steps)
    if "segmented" in legs:
        res["legs"]["segmented"] = segmented_leg(wr, ctx, args.steps)
        torch.cuda.empty_cache()
    if "wms" in legs:
        rs = [int(x) for x in args.wms_runs.split(",")]
        res["legs"]["wms"] = wms_leg(wr, ctx, rs[0], rs[1], max(1, args.steps // 5), 1, with_cpu,
                                     args.cpu_seconds)
        torch.cuda.empty_cache()
    rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
    if "serving" in legs and rates:
        res["serving"] = serving_leg(wr, ctx, rates, args.serve_seconds,
                                     [int(x) for x in args.serve_epochs.split(",") if x.strip()])
    if args.copy_probe > 0:
        n = args.copy_probe << 18
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = int(n) * 4
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
