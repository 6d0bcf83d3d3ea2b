// Batch planner and relaxation drivers behind wr_sssp / wr_order_matrices.
//
// Planning (host): distinct sources are solved once per call (many picks
// share vertices); they are ordered by tile and vertex id so that sources
// relaxed together sit close to each other, then cut into chunks whose work
// buffers fit the context's memory budget.  Each chunk is relaxed to the
// fixpoint by one of the schedules, then read out (rows, order matrices,
// predecessors) before the next chunk reuses the buffers.
//
// Pass loops run on device with device-side termination counters; a fixed
// number of passes is captured once in a hipGraph and replayed until a
// replay ends with nothing left to do (one host read per replay).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <numeric>
#include <sstream>

#include "wr_internal.hpp"

namespace wr {

// --------------------------------------------------------------- workspace
// Events around each relaxation-kernel launch of one replay (2 per pass).
struct KernelEvents {
    std::vector<hipEvent_t> ev;
    void create(uint32_t K) {
        ev.assign(2 * K, nullptr);
        for (auto &e : ev) WR_HIP(hipEventCreate(&e));
    }
    ~KernelEvents() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    hipEvent_t b(uint32_t i) const { return ev.empty() ? nullptr : ev[2 * i]; }
    hipEvent_t e(uint32_t i) const { return ev.empty() ? nullptr : ev[2 * i + 1]; }
    // Adds the K kernel durations of the replay that just finished; false if
    // the runtime cannot time these events (then nothing is added).
    bool collect(uint32_t K, wr_run_info &info) const {
        if (ev.empty()) return true;
        double sum = 0;
        for (uint32_t i = 0; i < K; ++i) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) {
                (void)hipGetLastError();
                return false;
            }
            sum += ms;
        }
        info.kernel_ms += sum;
        info.kernel_launches += K;
        return true;
    }
};

struct SegWork {
    uint64_t gen = 0;
    uint32_t S_cap = 0, tile_cap = 0, waves = 0, G = 0, K = 0, grid = 0, lanes = 1;   // S_cap: state rows
    bool timed = false;
    bool overlay = false;
    uint32_t grid_ovl = 0;
    KernelEvents kev;
    SegBuffers buf;
    hipGraphExec_t exec = nullptr;   // K passes of the segment kernel, or of the overlay kernel
    hipGraphExec_t exec2 = nullptr;  // overlay: 2 passes, to end a batch of replays near the expected count
    hipGraphExec_t exec_p = nullptr;  // overlay with target bounds (captured on first use)
    DBuf<uint32_t> bound, bound_tmp;  // target bounds per source slot and their refinement scratch
    SegState ss;
    // overlay: every exit value of all S_cap rows is INF (state_clean), else
    // the rows a call may have left dirty; a call that ends cleanly resets
    // its rows behind the host's wait, so the next call can skip the reset
    bool state_clean = false;
    uint32_t dirty_rows = 0;
    hipStream_t st = nullptr;        // stream the state's kernels run on
    ~SegWork() {
        if (st) (void)hipStreamSynchronize(st);   // a trailing reset may still run
        if (exec) (void)hipGraphExecDestroy(exec);
        if (exec2) (void)hipGraphExecDestroy(exec2);
        if (exec_p) (void)hipGraphExecDestroy(exec_p);
    }
};

struct BlkWork {
    uint32_t nb_cap = 0, K = 0, grid = 0;
    bool frontier = false;
    bool timed = false;
    KernelEvents kev;
    DBuf<uint32_t> dist, stamps, ctr, src;
    DBuf<uint64_t> list;
    DBuf<unsigned long long> stats;
    hipGraphExec_t exec = nullptr;
    ~BlkWork() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

struct Workspace {
    std::unique_ptr<SegWork> seg;
    std::unique_ptr<BlkWork> blk;
    uint32_t *h_flag = nullptr;   // pinned host word for termination checks
    // per-call index arrays of wr_order_matrices and the in-tile job, reused
    DBuf<uint32_t> call_off, call_picks, call_sidx;
    // source dedup: per-vertex stamp of the last call that saw it, its slot,
    // and the bucket counts of the source ordering
    std::vector<uint32_t> stamp, slot, plan_cnt;
    uint32_t stamp_id = 0;
    // passes the last segmented / overlay solve needed (replays launched
    // before the first convergence check), and how many of them had work
    uint64_t last_passes = 0, last_work_passes = 0;
    DBuf<uint64_t> call_base;
    IntileJob intile;
    hipEvent_t ev_done = nullptr;   // end of a call's results, ahead of a trailing reset
    // recorded about two thirds into a solve's first batch of replays, when
    // mid_valid: side-stream work that does not depend on the relaxation
    // waits for it, so it overlaps the light last passes, not the heavy first
    hipEvent_t ev_mid = nullptr;
    bool mid_valid = false;
    ~Workspace() {
        seg.reset();
        if (ev_done) (void)hipEventDestroy(ev_done);
        if (ev_mid) (void)hipEventDestroy(ev_mid);
        if (h_flag) (void)hipHostFree(h_flag);
    }
};

void destroy_workspace(Workspace *ws) { delete ws; }

namespace {

Workspace &workspace(wr_graph *g) {
    if (!g->ws) {
        g->ws = new Workspace();
        WR_HIP(hipHostMalloc(reinterpret_cast<void **>(&g->ws->h_flag), 64, hipHostMallocDefault));
    }
    return *g->ws;
}

// Host timeline of a call, printed to stderr when WR_TRACE is set.
struct CallTrace {
    bool on = std::getenv("WR_TRACE") != nullptr;
    double t0 = 0, last = 0;
    std::string line;
    void start(double t) {
        t0 = last = t;
        line.clear();
    }
    void mark(const char *what, double t) {
        if (!on) return;
        char b[64];
        std::snprintf(b, sizeof b, " %s %.3f", what, t - last);
        line += b;
        last = t;
    }
    void flush(const char *call) const {
        if (on) std::fprintf(stderr, "[wroute %s] ms:%s | total %.3f\n", call, line.c_str(), last - t0);
    }
};
CallTrace g_trace;

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

bool overlay_supported(const wr_graph *g) {
    const TileSet *ts = g->tiles;
    // every port has an incoming cross arc, so the arc bound also bounds the
    // ports (the in-tile tables hold 64 of them)
    return ts && g->lanes == 64 && g->max_w < 65536u && ts->max_cross_in <= ovl_max_entries() &&
           ts->max_exits <= ovl_max_exits() && ts->max_cross <= ovl_max_cross() &&
           (ts->tile_cap == 256 || ts->tile_cap == 512);
}

// The schedule of a call.  Segment-based schedules build the tile tables on
// first use; AUTO takes the overlay tables when the tiling allows them, the
// source-blocked segments otherwise, and the frontier when weights do not fit
// the 16-bit tile packing.
uint32_t resolve_algo(wr_graph *g, uint32_t flags) {
    uint32_t a = flags & WR_ALGO_MASK;
    switch (a) {
    case WR_ALGO_AUTO:
    case WR_ALGO_SWEEP:
    case WR_ALGO_FRONTIER:
    case WR_ALGO_SEGMENTED:
    case WR_ALGO_EDGE_B1:
    case WR_ALGO_EDGE_B0:
    case WR_ALGO_OVERLAY:
        break;
    default:
        fail(WR_E_INVALID, "unknown WR_ALGO value");
    }
    if ((a == WR_ALGO_SEGMENTED || a == WR_ALGO_OVERLAY) && g->max_w >= 65536u)
        fail(WR_E_UNSUPPORTED, "segment schedules pack weights in 16 bits; max weight is too large");
    if (a == WR_ALGO_AUTO && g->max_w >= 65536u) return WR_ALGO_FRONTIER;
    if (a == WR_ALGO_AUTO || a == WR_ALGO_SEGMENTED || a == WR_ALGO_OVERLAY) rebuild_tiles_if_needed(g);
    if (a == WR_ALGO_AUTO) a = overlay_supported(g) ? WR_ALGO_OVERLAY : WR_ALGO_SEGMENTED;
    if (a == WR_ALGO_OVERLAY && !overlay_supported(g))
        fail(WR_E_UNSUPPORTED, "the tiling does not fit the overlay tables (tiles of at most 512 "
                               "vertices with at most " + std::to_string(ovl_max_exits()) + " exits, " +
                               std::to_string(ovl_max_entries()) + " cross arcs entering and " +
                               std::to_string(ovl_max_cross()) + " leaving each)");
    return a;
}

// Distinct sources in processing order plus, for each requested vertex, its
// index among them.
struct Plan {
    std::vector<uint32_t> usrc;
    std::vector<uint32_t> uidx;
};

// Distinct sources of a call in block order, and each input's index among
// them.  Duplicates are found with a per-vertex stamp kept in the workspace
// and the order is a counting sort over tile ranks (sorting by vertex only
// inside a tile), so the cost is linear in the picks plus the tiles.
Plan make_plan(wr_graph *g, const uint32_t *verts, size_t n, bool by_tile) {
    Workspace &ws = workspace(g);
    if (ws.stamp.size() != g->V) {
        ws.stamp.assign(g->V, 0u);
        ws.slot.assign(g->V, 0u);
        ws.stamp_id = 0;
    }
    if (++ws.stamp_id == 0) {   // wrapped: clear the stamps
        std::fill(ws.stamp.begin(), ws.stamp.end(), 0u);
        ws.stamp_id = 1;
    }
    const uint32_t id = ws.stamp_id;
    Plan p;
    std::vector<uint32_t> &u = p.usrc;
    u.reserve(n);
    for (size_t k = 0; k < n; ++k) {
        const uint32_t v = verts[k];
        if (ws.stamp[v] == id) continue;
        ws.stamp[v] = id;
        u.push_back(v);
    }
    if (by_tile && g->tiles) {
        // blocks of 64 consecutive sources should start close together: a
        // counting sort by the tile's rank in key order (a compact patch
        // order for grid tilings; untiled vertices last), vertex id inside a
        // tile
        const TileSet &ts = *g->tiles;
        const std::vector<uint32_t> &rank = tile_order_rank(g);
        std::vector<uint32_t> &cnt = ws.plan_cnt;
        cnt.assign(static_cast<size_t>(ts.T) + 2, 0u);
        std::vector<uint32_t> rk(u.size());
        for (size_t i = 0; i < u.size(); ++i) {
            const uint32_t t = ts.tile_of[u[i]];
            rk[i] = t == NONE ? ts.T : rank[t];
            cnt[rk[i] + 1]++;
        }
        for (uint32_t r = 0; r <= ts.T; ++r) cnt[r + 1] += cnt[r];
        std::vector<uint32_t> sorted(u.size());
        for (size_t i = 0; i < u.size(); ++i) sorted[cnt[rk[i]]++] = u[i];
        // cnt[r] is now the end of bucket r; buckets are small
        uint32_t beg = 0;
        for (uint32_t r = 0; r <= ts.T; ++r) {
            const uint32_t end = cnt[r];
            if (end - beg > 1) std::sort(sorted.begin() + beg, sorted.begin() + end);
            beg = end;
        }
        u.swap(sorted);
    } else {
        std::sort(u.begin(), u.end());
    }
    for (uint32_t i = 0; i < u.size(); ++i) ws.slot[u[i]] = i;
    p.uidx.resize(n);
    for (size_t k = 0; k < n; ++k) p.uidx[k] = ws.slot[verts[k]];
    return p;
}

// -------------------------------------------------------- segmented driver
uint64_t seg_units_cap(const TileSet &ts, uint32_t S, uint32_t G) {
    return static_cast<uint64_t>(ts.T) * ((S + G - 1) / G) + ts.T;
}

}  // namespace

uint64_t SegBuffers::bytes_per_row(const TileSet &ts, uint32_t G, uint32_t lanes, bool overlay) {
    return 4ull * lanes * ((overlay ? ts.NB : ts.Vt + ts.NP) + 2) + 2ull * ts.T + 4ull * ts.T + 8ull * ts.T +
           8ull * ts.T / G + 8;
}

void SegBuffers::init(wr_context *ctx, const TileSet &ts, uint32_t S, uint32_t g, uint32_t ln, bool with_flags) {
    S_cap = S;
    G = g;
    lanes = ln;
    // the overlay schedule keeps the exits' values only
    if (with_flags) {
        xval.alloc(ctx, static_cast<size_t>(S) * std::max(ts.NB, 1u) * lanes);
    } else {
        gdist.alloc(ctx, static_cast<size_t>(S) * ts.Vt * lanes);
        inbox.alloc(ctx, static_cast<size_t>(S) * std::max(ts.NP, 1u) * lanes);
    }
    stamps.alloc(ctx, static_cast<size_t>(S) * ts.T);
    visited.alloc(ctx, static_cast<size_t>(S) * ts.T);
    if (with_flags) {
        flags.alloc(ctx, static_cast<size_t>(S) * ts.T);
        pending.alloc(ctx, S);
    }
    cnt.alloc(ctx, 2ull * ts.T);
    bucket.alloc(ctx, 2ull * ts.T * S);
    tiles.alloc(ctx, 2ull * ts.T);
    ctr.alloc(ctx, 8);
    // the overlay pass permutes unit indices with a prime above the count
    if (seg_units_cap(ts, S, G) >= 2654435761ull) fail(WR_E_NOMEM, "too many work units for one state");
    units.alloc(ctx, seg_units_cap(ts, S, G));
    stats.alloc(ctx, 2);
    if (with_flags) {
        // the overlay pass runs at most 4 workgroups of 8 waves per CU
        wave_slots = static_cast<uint32_t>(ctx->num_cus) * 32u;
        tile_visits.alloc(ctx, std::max(ts.T, 1u));
        wave_stores.alloc(ctx, wave_slots);
    }
    src_pos.alloc(ctx, static_cast<size_t>(S) * lanes);
    src_tile.alloc(ctx, static_cast<size_t>(S) * lanes);
    ss = SegState{};
    ss.S = S;
    ss.lanes_log2 = lanes == 64 ? 6u : 0u;
    ss.nsrc = S * lanes;
    ss.gdist = gdist.p;
    ss.inbox = inbox.p;
    ss.xval = xval.p;
    ss.visited = visited.p;
    ss.stamps = stamps.p;
    ss.cnt = cnt.p;
    ss.bucket = bucket.p;
    ss.tiles = tiles.p;
    ss.units = units.p;
    ss.ntiles = ctr.p + 0;   // [2]
    ss.nunits = ctr.p + 2;
    ss.cursor = ctr.p + 3;
    ss.pass_ctr = ctr.p + 4;
    ss.stats = stats.p;
    ss.src_pos = src_pos.p;
    ss.src_tile = src_tile.p;
    ss.flags = with_flags ? flags.p : nullptr;
    ss.pending = with_flags ? pending.p : nullptr;
    ss.tile_visits = with_flags ? tile_visits.p : nullptr;
    ss.wave_stores = with_flags ? wave_stores.p : nullptr;
}

uint32_t seg_pass_grid(const wr_context *ctx, uint32_t tile_cap, uint32_t waves, uint32_t lanes) {
    const uint32_t lds = seg_pass_lds_bytes(tile_cap, waves, lanes);
    uint32_t per_cu = std::max(1u, (160u * 1024u) / lds);
    per_cu = std::min(per_cu, 32u / waves);
    return static_cast<uint32_t>(ctx->num_cus) * per_cu;
}

// Captures K overlay passes starting at parity 1 (pass 0 of a chunk is the
// seed kernel over the sources' tiles), so a replay ends at parity 1.
hipGraphExec_t capture_ovl_passes(const TileSet &ts, const SegState &ss, uint32_t K, uint32_t G, uint32_t grid,
                                  const uint32_t *F, hipStream_t st, const uint32_t *bound) {
    hipGraph_t graph;
    WR_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
        for (uint32_t i = 0; i < K; ++i)
            launch_ovl_step(ts, ss, (i + 1) & 1u, G, grid, F, i + 1 == K, st, nullptr, nullptr, bound);
    } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(st, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
    }
    WR_HIP(hipStreamEndCapture(st, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) fail(WR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return exec;
}

hipGraphExec_t capture_seg_passes(const TileSet &ts, const SegState &ss, uint32_t K, uint32_t tile_cap,
                                  uint32_t waves, uint32_t G, uint32_t grid, hipStream_t st) {
    hipGraph_t graph;
    WR_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
        for (uint32_t i = 0; i < K; ++i) launch_seg_step(ts, ss, i & 1u, tile_cap, waves, G, grid, st);
    } catch (...) {
        hipGraph_t dummy = nullptr;
        (void)hipStreamEndCapture(st, &dummy);
        if (dummy) (void)hipGraphDestroy(dummy);
        throw;
    }
    WR_HIP(hipStreamEndCapture(st, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) fail(WR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return exec;
}

namespace {

// Boundary tables of the current weight epoch (computed on first use and
// after every weight update).
void ensure_overlay_tables(wr_graph *g) {
    TileSet &ts = *g->tiles;
    if (!ts.d_F.p) ts.d_F.alloc(g->ctx, static_cast<size_t>(ts.Vt) * 64);
    if (!ts.d_ovl_hdr.p) {
        // staging headers and per-exit arc offsets (fixed for the tiling)
        std::vector<uint32_t> &hdr = ts.ovl_hdr, &xb = ts.bo_xbeg;
        hdr.assign(4ull * ts.T, 0u);
        xb.assign(static_cast<size_t>(ts.NB) + ts.T, 0u);
        for (uint32_t t = 0; t < ts.T; ++t) {
            const uint32_t base = ts.tile_base[t], next = ts.tile_base[t + 1];
            const uint32_t p0 = ts.port_base[t], E = ts.port_base[t + 1] - p0;
            const uint32_t b0 = ts.bo_base[t], X = ts.bo_base[t + 1] - b0;
            const uint32_t xa0 = ts.x_off[base], na = ts.x_off[next] - xa0;
            hdr[4ull * t + 0] = p0;
            hdr[4ull * t + 1] = b0;
            hdr[4ull * t + 2] = xa0;
            hdr[4ull * t + 3] = E | (X << 8) | (na << 16);
            for (uint32_t j = 0; j < X; ++j) xb[b0 + t + j] = ts.x_off[base + ts.bo_local[b0 + j]] - xa0;
            xb[b0 + t + X] = na;
        }
        // pull form: incoming cross arcs per port with their source exits
        std::vector<uint32_t> xsrc_exit(ts.x_port.size(), NONE);
        for (uint32_t t = 0; t < ts.T; ++t)
            for (uint32_t b = ts.bo_base[t]; b < ts.bo_base[t + 1]; ++b) {
                const uint32_t pos = ts.tile_base[t] + ts.bo_local[b];
                for (uint32_t k = ts.x_off[pos]; k < ts.x_off[pos + 1]; ++k) xsrc_exit[k] = b;
            }
        ts.pin_off.assign(static_cast<size_t>(ts.NP) + 1, 0u);
        for (uint32_t p : ts.x_port) ts.pin_off[p + 1]++;
        for (uint32_t p = 0; p < ts.NP; ++p) ts.pin_off[p + 1] += ts.pin_off[p];
        ts.pin_xa.assign(ts.x_port.size(), 0u);
        ts.pin_exit.assign(ts.x_port.size(), 0u);
        ts.pin_lport.assign(ts.x_port.size(), 0u);
        {
            std::vector<uint32_t> fill(ts.pin_off.begin(), ts.pin_off.end() - 1);
            for (uint32_t k = 0; k < ts.x_port.size(); ++k) {
                const uint32_t p = ts.x_port[k];
                const uint32_t slot = fill[p]++;
                ts.pin_xa[slot] = k;
                ts.pin_exit[slot] = xsrc_exit[k];
                ts.pin_lport[slot] = p - ts.port_base[ts.x_tile[k]];
            }
        }
        ts.ovl_hdr2.assign(2ull * ts.T, 0u);
        for (uint32_t t = 0; t < ts.T; ++t) {
            ts.ovl_hdr2[2ull * t] = ts.pin_off[ts.port_base[t]];
            ts.ovl_hdr2[2ull * t + 1] = ts.pin_off[ts.port_base[t + 1]] - ts.pin_off[ts.port_base[t]];
        }
        upload(ts.d_pin_off, g->ctx, ts.pin_off, g->ctx->stream);
        upload(ts.d_pin_xa, g->ctx, ts.pin_xa, g->ctx->stream);
        upload(ts.d_pin_exit, g->ctx, ts.pin_exit, g->ctx->stream);
        upload(ts.d_pin_lport, g->ctx, ts.pin_lport, g->ctx->stream);
        upload(ts.d_ovl_hdr2, g->ctx, ts.ovl_hdr2, g->ctx->stream);
        ts.d_pin_rec.alloc(g->ctx, std::max<size_t>(1, ts.pin_xa.size()));
        upload(ts.d_ovl_hdr, g->ctx, hdr, g->ctx->stream);
        upload(ts.d_bo_xbeg, g->ctx, xb, g->ctx->stream);
        upload(ts.d_vert_of, g->ctx, ts.vert_of, g->ctx->stream);
        ts.d_B.alloc(g->ctx, static_cast<size_t>(ts.Vt) * 64);
        ts.ovl_em = ovl_row_entries(ts);
        ts.d_Fx.alloc(g->ctx, std::max<size_t>(1, static_cast<size_t>(ts.NB) * ts.ovl_em));
    }
    if (ts.custom_epoch == g->epoch) return;
    const uint32_t grid = static_cast<uint32_t>(g->ctx->num_cus) * 2;
    launch_ovl_custom(ts, ts.tile_cap, ts.d_F.p, grid, g->ctx->stream, false);
    launch_ovl_custom(ts, ts.tile_cap, ts.d_B.p, grid, g->ctx->stream, true);
    launch_ovl_pack(ts, g->ctx->stream);
    launch_ovl_pin_rec(ts, g->ctx->stream);
    ts.custom_epoch = g->epoch;
}

SegWork &seg_workspace(wr_graph *g, uint32_t S_need, bool graph_mode, bool timed, bool overlay) {
    Workspace &ws = workspace(g);
    TileSet &ts = *g->tiles;
    const uint32_t waves = g->waves_per_group;
    const uint32_t lanes = g->lanes;
    const uint32_t G = g->sources_per_unit ? g->sources_per_unit : (lanes == 64 ? 4 : 4 * waves);
    const uint32_t K = std::max(2u, g->passes_per_replay & ~1u);
    const uint32_t rows_need = (S_need + lanes - 1) / lanes;
    SegWork *w = ws.seg.get();
    const bool fits = w && w->gen == g->tiles_gen && w->S_cap >= rows_need && w->tile_cap == ts.tile_cap &&
                      w->waves == waves && w->lanes == lanes && w->G == G && w->K == K &&
                      w->timed == timed && w->overlay == overlay && (!graph_mode || w->exec);
    if (fits) return *w;
    // size the chunk: the request, bounded by the budget (keep what we hold;
    // the overlay's epoch tables are allocated first, the state takes the rest)
    ws.seg.reset();
    if (overlay) ensure_overlay_tables(g);
    const uint64_t per = SegBuffers::bytes_per_row(ts, G, lanes, overlay);
    const uint64_t avail = g->ctx->available();
    uint64_t R_fit = avail > (64ull << 20) ? (avail - (64ull << 20)) / per : 0;
    uint32_t R_cap = static_cast<uint32_t>(std::min<uint64_t>(rows_need, R_fit));
    if (R_cap == 0) fail(WR_E_NOMEM, "not even one source fits the memory budget (segmented)");
    auto nw = std::make_unique<SegWork>();
    nw->st = g->ctx->stream;
    nw->gen = g->tiles_gen;
    nw->S_cap = R_cap;
    nw->tile_cap = ts.tile_cap;
    nw->waves = waves;
    nw->lanes = lanes;
    nw->G = G;
    nw->K = K;
    nw->timed = timed;
    nw->overlay = overlay;
    if (timed) nw->kev.create(K);
    wr_context *ctx = g->ctx;
    nw->buf.init(ctx, ts, R_cap, G, lanes, overlay);
    nw->ss = nw->buf.ss;
    nw->grid = seg_pass_grid(ctx, ts.tile_cap, waves, lanes);
    nw->grid_ovl = static_cast<uint32_t>(ctx->num_cus) *
                   std::min(32u / ovl_waves(), std::max(1u, (160u * 1024u) / ovl_pass_lds_bytes(ts)));
    if (overlay) ensure_overlay_tables(g);
    if (overlay) {
        nw->bound.alloc(ctx, static_cast<size_t>(R_cap) * lanes);
        nw->bound_tmp.alloc(ctx, static_cast<size_t>(R_cap) * lanes);
    }
    if (graph_mode)
        nw->exec2 = overlay ? capture_ovl_passes(ts, nw->ss, 2, G, nw->grid_ovl, ts.d_F.p, ctx->stream, nullptr)
                            : nullptr;
    if (graph_mode)
        nw->exec = overlay ? capture_ovl_passes(ts, nw->ss, K, G, nw->grid_ovl, ts.d_F.p, ctx->stream, nullptr)
                           : capture_seg_passes(ts, nw->ss, K, ts.tile_cap, waves, G, nw->grid, ctx->stream);
    ws.seg = std::move(nw);
    return *ws.seg;
}

// Relaxes sources usrc[lo .. lo+n) to the fixpoint in the segmented state.
// `overlap` (may be empty) runs on the host once the first passes are on the
// GPU, so host work of the caller overlaps the relaxation.
void seg_solve_chunk(wr_graph *g, SegWork &w, const std::vector<uint32_t> &usrc, uint32_t lo,
                     uint32_t n, bool graph_mode, wr_run_info &info, const std::function<void()> &overlap,
                     const std::function<void()> &refine) {
    const TileSet &ts = *g->tiles;
    wr_context *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    SegState ss = w.ss;
    // per-source tables, padded with NONE up to the state's capacity
    const uint32_t lanes = w.lanes;
    const uint32_t rows = (n + lanes - 1) / lanes;
    const size_t cap_src = static_cast<size_t>(w.S_cap) * lanes;
    std::vector<uint32_t> sp(cap_src, NONE), stl(cap_src, NONE);
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t v = usrc[lo + i];
        sp[i] = ts.pos_of[v];
        stl[i] = ts.tile_of[v];
    }
    WR_HIP(hipMemcpyAsync(w.buf.src_pos.p, sp.data(), cap_src * 4, hipMemcpyHostToDevice, st));
    WR_HIP(hipMemcpyAsync(w.buf.src_tile.p, stl.data(), cap_src * 4, hipMemcpyHostToDevice, st));
    // reset the chunk state (the layout keeps the capacity for indexing)
    if (w.overlay) {
        if (!w.state_clean)
            launch_fill_u32(w.buf.xval.p, static_cast<size_t>(w.S_cap) * std::max(ts.NB, 1u) * lanes, INF, st);
        w.state_clean = false;
        w.dirty_rows = rows;
    } else
        launch_fill_u32(w.buf.inbox.p, static_cast<size_t>(rows) * std::max(ts.NP, 1u) * lanes, INF, st);
    launch_fill_u32(w.buf.stamps.p, static_cast<size_t>(rows) * ts.T, 0u, st);
    launch_fill_u8(w.buf.visited.p, static_cast<size_t>(rows) * ts.T, 0u, st);
    if (w.overlay) {
        // flags are [tile][row]: clear every row of the state, which also
        // drops flags an aborted earlier solve may have left
        launch_fill_u8(w.buf.flags.p, static_cast<size_t>(w.S_cap) * ts.T, 0u, st);
        launch_fill_u32(w.buf.tile_visits.p, std::max(ts.T, 1u), 0u, st);
        launch_fill_u32(w.buf.wave_stores.p, w.buf.wave_slots, 0u, st);
    }
    launch_fill_u32(w.buf.cnt.p, 2ull * ts.T, 0u, st);
    launch_fill_u32(w.buf.ctr.p, 8, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t *>(w.buf.stats.p), 4, 0u, st);
    // target-bounded passes (refine set): bounds start unlimited and shrink
    // after every replay; the bounded passes are captured on first use
    const bool bounded = w.overlay && static_cast<bool>(refine);
    // bounded solves replay short graphs so the bounds tighten early
    const uint32_t Kb = std::min<uint32_t>(w.K, 4u);
    if (bounded) {
        launch_fill_u32(w.bound.p, cap_src, INF, st);
        launch_fill_u32(w.bound_tmp.p, cap_src, 0u, st);
        if (graph_mode && !w.exec_p)
            w.exec_p = capture_ovl_passes(ts, ss, Kb, w.G, w.grid_ovl, ts.d_F.p, st, w.bound.p);
    }
    g_trace.mark("chunk_reset", now_ms());
    if (!w.overlay) launch_seg_seed_n(ts, ss, n, st);
    hipEvent_t e0, e1;
    WR_HIP(hipEventCreate(&e0));
    WR_HIP(hipEventCreate(&e1));
    WR_HIP(hipEventRecord(e0, st));
    const uint32_t K = bounded ? Kb : w.K;   // passes per replay
    uint64_t passes = 0;
    const uint64_t cap = static_cast<uint64_t>(g->V) + 2ull * K + 8;
    // overlay: pass 0 stores the sources' in-tile exit distances (the seed
    // kernel); the replayed passes then start at parity 1 and end there
    const uint32_t par0 = w.overlay ? 1u : 0u;
    if (w.overlay) {
        if (ts.custom_epoch != g->epoch) ensure_overlay_tables(g);
        launch_ovl_seed_push(ts, ss, nullptr, rows * 64, st);
        passes += 1;
    }
    // replays launched before the first convergence check: as many as the
    // previous solve needed (surplus passes find nothing to do and are cheap)
    Workspace &wsp = workspace(g);
    uint32_t batch = graph_mode ? static_cast<uint32_t>(std::max<uint64_t>(1, wsp.last_passes / K)) : 1u;
    // overlay: cover the previous solve's passes with work by K-pass replays
    // plus 2-pass ones, so the first check comes at most one pass late
    // (bounded passes refine their bounds after every replay instead)
    if (bounded) batch = 1;
    uint32_t batch2 = 0;
    if (graph_mode && w.exec2 && wsp.last_work_passes > 0 && !bounded) {
        batch = static_cast<uint32_t>(wsp.last_work_passes / K);
        batch2 = static_cast<uint32_t>((wsp.last_work_passes - static_cast<uint64_t>(batch) * K + 1) / 2);
    }
    bool first = true;
    wsp.mid_valid = false;
    for (;;) {
        if (graph_mode) {
            const uint32_t mid = first && overlap && batch >= 2 ? (2 * batch + 2) / 3 : batch;
            for (uint32_t r = 0; r < batch; ++r) {
                if (r == mid) {
                    if (!wsp.ev_mid) WR_HIP(hipEventCreateWithFlags(&wsp.ev_mid, hipEventDisableTiming));
                    WR_HIP(hipEventRecord(wsp.ev_mid, st));
                    wsp.mid_valid = true;
                }
                WR_HIP(hipGraphLaunch(bounded ? w.exec_p : w.exec, st));
            }
            for (uint32_t r = 0; r < batch2; ++r) WR_HIP(hipGraphLaunch(w.exec2, st));
            if (batch + batch2 == 0) {
                WR_HIP(hipGraphLaunch(bounded ? w.exec_p : w.exec, st));
                batch = 1;
            }
            passes += static_cast<uint64_t>(K) * batch + 2ull * batch2;
            batch = 1;
            batch2 = 0;
        } else if (w.overlay) {
            for (uint32_t i = 0; i < K; ++i)
                launch_ovl_step(ts, ss, (i + 1) & 1u, w.G, w.grid_ovl, ts.d_F.p, i + 1 == K, st, w.kev.b(i),
                                w.kev.e(i), bounded ? w.bound.p : nullptr);
            passes += K;
        } else {
            for (uint32_t i = 0; i < K; ++i)
                launch_seg_step(ts, ss, i & 1u, ts.tile_cap, w.waves, w.G, w.grid, st, w.kev.b(i),
                                w.kev.e(i));
            passes += K;
        }
        if (bounded) refine();
        if (first && overlap) overlap();
        first = false;
        WR_HIP(hipMemcpyAsync(workspace(g).h_flag, ss.ntiles + par0, 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipStreamSynchronize(st));
        if (!w.kev.collect(K, info)) fail(WR_E_DEVICE, "kernel event timing failed");
        if (*workspace(g).h_flag == 0) break;
        if (passes > cap) fail(WR_E_INTERNAL, "segmented relaxation exceeded its pass cap");
    }
    g_trace.mark("replays", now_ms());
    wsp.last_passes = passes;
    WR_HIP(hipEventRecord(e1, st));
    unsigned long long stats[2];
    WR_HIP(hipMemcpyAsync(stats, w.buf.stats.p, sizeof(stats), hipMemcpyDeviceToHost, st));
    std::vector<uint32_t> tv, wsr;
    if (w.overlay) {
        tv.resize(std::max(ts.T, 1u));
        wsr.resize(w.buf.wave_slots);
        WR_HIP(hipMemcpyAsync(tv.data(), w.buf.tile_visits.p, tv.size() * 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipMemcpyAsync(wsr.data(), w.buf.wave_stores.p, wsr.size() * 4, hipMemcpyDeviceToHost, st));
    }
    WR_HIP(hipStreamSynchronize(st));
    float ms = 0;
    WR_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    info.relax_ms += ms;
    info.passes += static_cast<uint32_t>(stats[1]);
    if (!w.overlay) info.work_items += stats[0];
    if (w.overlay) {
        wsp.last_work_passes = stats[1];
        // a visit of tile t reads a 256-byte row per incoming cross arc and
        // per exit, and relaxes its incoming arcs and its exits' table
        // entries for 64 lanes; every stored exit value writes 4 bytes
        uint64_t rows_read = 0, relax = 0, stored = 0;
        for (uint32_t t = 0; t < ts.T; ++t) {
            const uint64_t hw = ts.ovl_hdr[4ull * t + 3], E = hw & 0xFFu, X = (hw >> 8) & 0xFFu;
            const uint64_t npa = ts.ovl_hdr2[2ull * t + 1];
            rows_read += tv[t] * (npa + X);
            relax += tv[t] * (npa + E * X);
        }
        for (uint32_t v : wsr) stored += v;
        uint64_t visits = 0;
        for (uint32_t t = 0; t < ts.T; ++t) visits += tv[t];
        info.work_items += visits;
        info.relaxations += 64ull * relax;
        info.alg_bytes += 256ull * rows_read + 4ull * stored;
    }
}

// ------------------------------------------------------ blocked-layout driver
uint64_t blk_bytes_per_block(uint32_t V, bool frontier) {
    return static_cast<uint64_t>(V) * (LANES * 4ull + (frontier ? 4ull + 16ull : 0ull));
}

// One replay's worth of passes of the blocked-layout schedule (captured or
// eager): K frontier passes, or a cleared changed-flag and K sweeps.
void blk_passes(wr_graph *g, BlkWork &w, hipStream_t st) {
    const size_t units = static_cast<size_t>(w.nb_cap) * g->V;
    if (w.frontier) {
        for (uint32_t i = 0; i < w.K; ++i) {
            const uint32_t par = i & 1u, nx = par ^ 1u;
            launch_pass_prologue(w.ctr.p + nx, w.ctr.p + par, w.stats.p, w.ctr.p + 4, st);
            if (w.kev.b(i)) WR_HIP(hipEventRecord(w.kev.b(i), st));
            launch_frontier_push(w.dist.p, g->V, g->d_row_ptr.p, g->d_col.p, g->d_w.p,
                                 w.list.p + par * units, w.ctr.p + par, w.list.p + nx * units,
                                 w.ctr.p + nx, w.stamps.p, w.ctr.p + 4, w.grid, st);
            if (w.kev.e(i)) WR_HIP(hipEventRecord(w.kev.e(i), st));
        }
    } else {
        launch_fill_u32(w.ctr.p + 2, 1, 0u, st);
        for (uint32_t i = 0; i < w.K; ++i) {
            if (w.kev.b(i)) WR_HIP(hipEventRecord(w.kev.b(i), st));
            launch_sweep_pull(w.dist.p, g->V, w.nb_cap, g->d_in_ptr.p, g->d_in_src.p, g->d_in_w.p,
                              w.ctr.p + 2, w.grid, st);
            if (w.kev.e(i)) WR_HIP(hipEventRecord(w.kev.e(i), st));
        }
    }
}

BlkWork &blk_workspace(wr_graph *g, uint32_t nb_need, bool frontier, bool graph_mode, bool timed) {
    Workspace &ws = workspace(g);
    const uint32_t K = std::max(2u, g->passes_per_replay & ~1u);
    BlkWork *w = ws.blk.get();
    if (w && w->nb_cap >= nb_need && w->frontier == frontier && w->K == K && w->timed == timed &&
        (!graph_mode || w->exec))
        return *w;
    ws.blk.reset();
    const uint64_t per = blk_bytes_per_block(g->V, frontier);
    const uint64_t avail = g->ctx->available();
    uint64_t nb_fit = avail > (64ull << 20) ? (avail - (64ull << 20)) / per : 0;
    const uint32_t nb_cap = static_cast<uint32_t>(std::min<uint64_t>(nb_need, nb_fit));
    if (nb_cap == 0) fail(WR_E_NOMEM, "not even one source block fits the memory budget");
    auto nw = std::make_unique<BlkWork>();
    nw->nb_cap = nb_cap;
    nw->frontier = frontier;
    nw->K = K;
    nw->timed = timed;
    if (timed) nw->kev.create(K);
    wr_context *ctx = g->ctx;
    const size_t units = static_cast<size_t>(nb_cap) * g->V;
    nw->dist.alloc(ctx, units * LANES);
    nw->ctr.alloc(ctx, 8);
    nw->src.alloc(ctx, static_cast<size_t>(nb_cap) * LANES);
    nw->stats.alloc(ctx, 2);
    if (frontier) {
        nw->stamps.alloc(ctx, units);
        nw->list.alloc(ctx, 2 * units);
    }
    nw->grid = static_cast<uint32_t>(ctx->num_cus) * 8;
    if (graph_mode) {
        hipStream_t st = ctx->stream;
        hipGraph_t graph;
        WR_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        try {
            blk_passes(g, *nw, st);
        } catch (...) {
            hipGraph_t dummy;
            (void)hipStreamEndCapture(st, &dummy);
            if (dummy) (void)hipGraphDestroy(dummy);
            throw;
        }
        WR_HIP(hipStreamEndCapture(st, &graph));
        hipError_t e = hipGraphInstantiate(&nw->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) fail(WR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    ws.blk = std::move(nw);
    return *ws.blk;
}

// Relaxes usrc[lo .. lo+n) in the blocked layout (n <= nb_cap * 64).  The
// sweep graph spans all nb_cap blocks; unused lanes stay INF and cost only
// bandwidth.
void blk_solve_chunk(wr_graph *g, BlkWork &w, const std::vector<uint32_t> &usrc, uint32_t lo,
                     uint32_t n, bool graph_mode, wr_run_info &info) {
    wr_context *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t V = g->V;
    const size_t units = static_cast<size_t>(w.nb_cap) * V;
    WR_HIP(hipMemcpyAsync(w.src.p, usrc.data() + lo, n * 4ull, hipMemcpyHostToDevice, st));
    launch_fill_u32(w.dist.p, units * LANES, INF, st);
    launch_fill_u32(w.ctr.p, 8, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t *>(w.stats.p), 4, 0u, st);
    launch_blk_seed(w.dist.p, V, n, w.src.p, st);
    if (w.frontier) {
        launch_fill_u32(w.stamps.p, units, 0u, st);
        launch_frontier_seed(w.list.p, w.ctr.p + 0, n, w.src.p, V, st);
    }
    hipEvent_t e0, e1;
    WR_HIP(hipEventCreate(&e0));
    WR_HIP(hipEventCreate(&e1));
    WR_HIP(hipEventRecord(e0, st));
    const uint32_t K = w.K;
    uint64_t passes = 0, sweeps_changed = 0;
    const uint64_t cap = static_cast<uint64_t>(V) + 2ull * K + 8;
    uint32_t *hf = workspace(g).h_flag;
    for (;;) {
        if (graph_mode)
            WR_HIP(hipGraphLaunch(w.exec, st));
        else
            blk_passes(g, w, st);
        passes += K;
        WR_HIP(hipMemcpyAsync(hf, w.frontier ? w.ctr.p + 0 : w.ctr.p + 2, 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipStreamSynchronize(st));
        if (!w.kev.collect(K, info)) fail(WR_E_DEVICE, "kernel event timing failed");
        if (!w.frontier && *hf) sweeps_changed += K;
        if (*hf == 0) break;
        if (passes > cap) fail(WR_E_INTERNAL, "relaxation exceeded its pass cap");
    }
    WR_HIP(hipEventRecord(e1, st));
    unsigned long long stats[2] = {0, 0};
    WR_HIP(hipMemcpyAsync(stats, w.stats.p, sizeof(stats), hipMemcpyDeviceToHost, st));
    WR_HIP(hipStreamSynchronize(st));
    float ms = 0;
    WR_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    info.relax_ms += ms;
    if (w.frontier) {
        info.passes += static_cast<uint32_t>(stats[1]);
        info.work_items += stats[0];
    } else {
        info.passes += static_cast<uint32_t>(passes);
        info.work_items += passes * units;
    }
    (void)sweeps_changed;
}

// --------------------------------------------------- edge-list baseline
// Runs the N sources of `src` together (dist [N][V]), one launch per round
// and a host read of the changed flag after each round (the paper's
// structure: a global synchronisation every iteration).  full_rounds runs
// exactly V-1 rounds.
void edge_solve(wr_graph *g, const uint32_t *d_src, uint32_t N, uint32_t *d_rows, bool full_rounds,
                wr_run_info &info) {
    wr_context *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t V = g->V;
    if (!g->d_arc_src.p && g->E) {
        g->d_arc_src.alloc(ctx, g->E);
        launch_arc_src(g->d_row_ptr.p, V, g->d_arc_src.p, st);
    }
    Workspace &ws = workspace(g);
    launch_fill_u32(d_rows, static_cast<size_t>(N) * V, INF, st);
    launch_rows_seed(d_rows, V, N, d_src, st);
    DBuf<uint32_t> flag;
    flag.alloc(ctx, 1);
    hipEvent_t e0, e1;
    WR_HIP(hipEventCreate(&e0));
    WR_HIP(hipEventCreate(&e1));
    WR_HIP(hipEventRecord(e0, st));
    const uint32_t rounds_cap = V > 1 ? V - 1 : 1;
    uint32_t rounds = 0;
    for (; rounds < rounds_cap;) {
        launch_fill_u32(flag.p, 1, 0u, st);
        launch_edge_round(g->d_arc_src.p, g->d_col.p, g->d_w.p, g->E, d_rows, V, N, flag.p, st);
        ++rounds;
        WR_HIP(hipMemcpyAsync(ws.h_flag, flag.p, 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipStreamSynchronize(st));
        if (!full_rounds && *ws.h_flag == 0) break;
    }
    WR_HIP(hipEventRecord(e1, st));
    WR_HIP(hipStreamSynchronize(st));
    float ms = 0;
    WR_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    info.relax_ms += ms;
    info.passes += rounds;
    info.work_items += static_cast<uint64_t>(rounds) * g->E;
}

// Orders `lo..lo+n)` of usrc that fit one chunk of the chosen schedule.
uint32_t chunk_sources(wr_graph *g, uint32_t algo, uint32_t total, bool graph_mode, bool timed) {
    if (algo == WR_ALGO_SEGMENTED || algo == WR_ALGO_OVERLAY) {
        SegWork &w = seg_workspace(g, total, graph_mode, timed, algo == WR_ALGO_OVERLAY);
        return w.S_cap * w.lanes;
    }
    const uint32_t nb_need = (total + LANES - 1) / LANES;
    return blk_workspace(g, nb_need, algo == WR_ALGO_FRONTIER, graph_mode, timed).nb_cap * LANES;
}

void solve_chunk(wr_graph *g, uint32_t algo, const std::vector<uint32_t> &usrc, uint32_t lo,
                 uint32_t n, bool graph_mode, wr_run_info &info,
                 const std::function<void()> &overlap = std::function<void()>(),
                 const std::function<void()> &refine = std::function<void()>()) {
    if (algo == WR_ALGO_SEGMENTED || algo == WR_ALGO_OVERLAY) {
        seg_solve_chunk(g, *workspace(g).seg, usrc, lo, n, graph_mode, info, overlap, refine);
    } else {
        blk_solve_chunk(g, *workspace(g).blk, usrc, lo, n, graph_mode, info);
        if (overlap) overlap();
    }
}

// Source-major rows of the current chunk's state: out + out_row[r]*V gets the
// row of chunk source row_idx[r].
void emit_rows(wr_graph *g, uint32_t algo, uint32_t rows, const uint32_t *d_row_idx,
               const uint32_t *d_row_vertex, const uint32_t *d_out_row, uint32_t *out,
               const std::vector<uint32_t> &row_idx, const std::vector<uint32_t> &row_vertex,
               const std::vector<uint32_t> &out_row);

// Index arrays given as device pointers (WR_DEVICE_INDEX): read back on the
// caller's stream, so the values its earlier work wrote are the ones read.
std::vector<uint32_t> fetch_index(const uint32_t *d, size_t n, void *stream) {
    std::vector<uint32_t> h(n);
    if (!n) return h;
    if (!d) fail(WR_E_INVALID, "an index array is NULL");
    hipStream_t us = static_cast<hipStream_t>(stream);
    WR_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(uint32_t), hipMemcpyDeviceToHost, us));
    WR_HIP(hipStreamSynchronize(us));
    return h;
}

struct StreamJoin {
    // The library works on its own stream; with caller (device) buffers it
    // first waits for the caller's stream so earlier work on them is done.
    StreamJoin(wr_context *ctx, bool dev, void *user_stream) {
        if (!dev) return;
        hipEvent_t ev;
        WR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        WR_HIP(hipEventRecord(ev, static_cast<hipStream_t>(user_stream)));
        WR_HIP(hipStreamWaitEvent(ctx->stream, ev, 0));
        (void)hipEventDestroy(ev);
    }
};

// Overlay read-outs hold paths that leave the source's tile; these add the
// in-tile distances of the source's own tile (groups of up to 64 sources of
// one tile).  Full rows: every vertex of the tile of each row's source.
IntileWork intile_rows(const TileSet &ts, const std::vector<uint32_t> &src_vertex,
                       const std::vector<uint32_t> &out_row) {
    std::map<uint32_t, std::vector<uint32_t>> by_tile;
    for (uint32_t i = 0; i < src_vertex.size(); ++i) {
        const uint32_t t = ts.tile_of[src_vertex[i]];
        if (t != NONE) by_tile[t].push_back(i);
    }
    IntileWork w;
    for (auto &kv : by_tile) {
        const uint32_t t = kv.first;
        for (size_t c = 0; c < kv.second.size(); c += 64) {
            const uint32_t nl = static_cast<uint32_t>(std::min<size_t>(64, kv.second.size() - c));
            w.grp.insert(w.grp.end(), {t, nl, 0u, 0u});
            for (uint32_t l = 0; l < 64; ++l) {
                const uint32_t i = l < nl ? kv.second[c + l] : kv.second[c];
                w.src_local.push_back(ts.pos_of[src_vertex[i]] - ts.tile_base[t]);
                w.row.push_back(out_row[i]);
            }
        }
    }
    return w;
}

// Order matrices: the entries (i, j) whose picks lie in one tile, for the
// picks whose source index passes `take` (out index = out_base[o] + i*P + j).
template <class Take>
IntileWork intile_pairs(const TileSet &ts, uint32_t num_orders, const uint32_t *off, const uint32_t *picks,
                        const uint64_t *out_base, Take take) {
    struct Entry {
        uint32_t t, src, tgt;
        uint64_t out;
    };
    std::vector<Entry> e;
    std::vector<std::pair<uint32_t, uint32_t>> by;   // (tile, index in the order)
    for (uint32_t o = 0; o < num_orders; ++o) {
        const uint32_t a = off[o], P = off[o + 1] - a;
        by.clear();
        for (uint32_t i = 0; i < P; ++i) {
            const uint32_t t = ts.tile_of[picks[a + i]];
            if (t != NONE) by.push_back({t, i});
        }
        std::sort(by.begin(), by.end());
        // pairs only within runs of one tile
        for (size_t r0 = 0; r0 < by.size();) {
            size_t r1 = r0 + 1;
            while (r1 < by.size() && by[r1].first == by[r0].first) ++r1;
            const uint32_t t = by[r0].first;
            for (size_t x = r0; x < r1; ++x) {
                const uint32_t i = by[x].second, si = picks[a + i];
                if (!take(a + i)) continue;
                for (size_t y = r0; y < r1; ++y) {
                    const uint32_t j = by[y].second, v = picks[a + j];
                    if (v == si) continue;
                    e.push_back({t, si, ts.pos_of[v] - ts.tile_base[t], out_base[o] + static_cast<uint64_t>(i) * P + j});
                }
            }
            r0 = r1;
        }
    }
    // order by (tile, source): a counting sort by tile, then each tile's
    // (short) run by source
    {
        std::vector<uint32_t> cnt(static_cast<size_t>(ts.T) + 1, 0u);
        for (const Entry &x : e) cnt[x.t + 1]++;
        for (uint32_t t = 0; t < ts.T; ++t) cnt[t + 1] += cnt[t];
        std::vector<Entry> sorted(e.size());
        std::vector<uint32_t> fill(cnt.begin(), cnt.end() - 1);
        for (const Entry &x : e) sorted[fill[x.t]++] = x;
        for (uint32_t t = 0; t < ts.T; ++t)
            if (cnt[t + 1] - cnt[t] > 1)
                std::sort(sorted.begin() + cnt[t], sorted.begin() + cnt[t + 1],
                          [](const Entry &x, const Entry &y) { return x.src < y.src; });
        e.swap(sorted);
    }
    IntileWork w;
    size_t k = 0;
    while (k < e.size()) {
        // one group: up to 64 distinct sources of tile e[k].t
        const uint32_t t = e[k].t;
        const size_t g0 = w.pair_key.size();
        std::vector<uint32_t> lanes;
        while (k < e.size() && e[k].t == t) {
            if (lanes.empty() || lanes.back() != e[k].src) {
                if (lanes.size() == 64) break;
                lanes.push_back(e[k].src);
            }
            w.pair_key.push_back((static_cast<uint32_t>(lanes.size() - 1) << 16) | e[k].tgt);
            w.pair_out.push_back(e[k].out);
            ++k;
        }
        const uint32_t nl = static_cast<uint32_t>(lanes.size());
        w.grp.insert(w.grp.end(), {t, nl, static_cast<uint32_t>(g0), static_cast<uint32_t>(w.pair_key.size())});
        for (uint32_t l = 0; l < 64; ++l) w.src_local.push_back(ts.pos_of[lanes[l < nl ? l : 0]] - ts.tile_base[t]);
    }
    return w;
}

void emit_rows(wr_graph *g, uint32_t algo, uint32_t rows, const uint32_t *d_row_idx,
               const uint32_t *d_row_vertex, const uint32_t *d_out_row, uint32_t *out,
               const std::vector<uint32_t> &row_idx, const std::vector<uint32_t> &row_vertex,
               const std::vector<uint32_t> &out_row) {
    hipStream_t st = g->ctx->stream;
    if (algo == WR_ALGO_OVERLAY) {
        SegWork &w = *workspace(g).seg;
        // row groups: per block of 64 chunk sources, the output row of each
        // lane; a source asked for twice takes a second group of its block
        std::vector<uint32_t> gblock, lrow;
        std::map<uint32_t, std::vector<uint32_t>> groups_of;
        for (uint32_t r = 0; r < rows; ++r) {
            const uint32_t sidx = row_idx[r], b = sidx >> 6, l = sidx & 63u;
            std::vector<uint32_t> &gs = groups_of[b];
            uint32_t gi = NONE;
            for (uint32_t x : gs)
                if (lrow[static_cast<size_t>(x) * 64 + l] == NONE) {
                    gi = x;
                    break;
                }
            if (gi == NONE) {
                gi = static_cast<uint32_t>(gblock.size());
                gblock.push_back(b);
                lrow.resize(lrow.size() + 64, NONE);
                gs.push_back(gi);
            }
            lrow[static_cast<size_t>(gi) * 64 + l] = out_row[r];
        }
        DBuf<uint32_t> d_gblock, d_lrow;
        upload(d_gblock, g->ctx, gblock, st);
        upload(d_lrow, g->ctx, lrow, st);
        launch_ovl_emit(*g->tiles, w.ss, g->tiles->d_F.p, g->V, rows, d_row_vertex, d_out_row, d_gblock.p, d_lrow.p,
                        static_cast<uint32_t>(gblock.size()), static_cast<uint32_t>(g->ctx->num_cus), out, st);
        launch_intile_fix(g->ctx, *g->tiles, intile_rows(*g->tiles, row_vertex, out_row), true, g->V, out, st);
    } else if (algo == WR_ALGO_SEGMENTED) {
        SegWork &w = *workspace(g).seg;
        launch_seg_emit(*g->tiles, w.ss, g->V, rows, d_row_idx, d_row_vertex, d_out_row, out, st);
    } else {
        BlkWork &w = *workspace(g).blk;
        launch_blk_emit(w.dist.p, g->V, rows, d_row_idx, d_out_row, out, st);
    }
}

}  // namespace

// ------------------------------------------------------ streaming overlay
struct StreamSolver {
    wr_graph *g = nullptr;
    uint64_t gen = 0;
    uint32_t blocks = 0;
};

namespace {

SegWork &stream_work(StreamSolver *s) {
    SegWork &w = seg_workspace(s->g, s->blocks * 64u, true, false, true);
    if (w.gen != s->gen || w.S_cap < s->blocks)
        fail(WR_E_INTERNAL, "the streaming state was rebuilt while requests were in flight");
    return w;
}

}  // namespace

uint64_t stream_bytes_per_block(wr_graph *g) {
    (void)resolve_algo(g, WR_ALGO_OVERLAY);
    return SegBuffers::bytes_per_row(*g->tiles, 4, 64, true);
}

StreamSolver *stream_create(wr_graph *g, uint32_t blocks) {
    (void)hipSetDevice(g->ctx->device);
    (void)resolve_algo(g, WR_ALGO_OVERLAY);
    if (!blocks) fail(WR_E_NOMEM, "no block row fits the memory budget");
    SegWork &w = seg_workspace(g, blocks * 64u, true, false, true);
    w.state_clean = false;   // rows are reset one by one at admission
    const TileSet &ts = *g->tiles;
    hipStream_t st = g->ctx->stream;
    launch_fill_u8(w.buf.flags.p, static_cast<size_t>(w.S_cap) * ts.T, 0u, st);
    launch_fill_u32(w.buf.pending.p, w.S_cap, 0u, st);
    launch_fill_u32(w.buf.cnt.p, 2ull * ts.T, 0u, st);
    launch_fill_u32(w.buf.ctr.p, 8, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t *>(w.buf.stats.p), 4, 0u, st);
    launch_fill_u32(w.buf.tile_visits.p, std::max(ts.T, 1u), 0u, st);
    launch_fill_u32(w.buf.wave_stores.p, w.buf.wave_slots, 0u, st);
    g_trace.mark("chunk_reset", now_ms());
    launch_fill_u32(w.buf.src_tile.p, static_cast<size_t>(w.S_cap) * 64, NONE, st);
    ensure_overlay_tables(g);
    WR_HIP(hipStreamSynchronize(st));
    auto *s = new StreamSolver();
    s->g = g;
    s->gen = w.gen;
    s->blocks = w.S_cap;
    return s;
}

void stream_destroy(StreamSolver *s) { delete s; }

uint32_t stream_blocks(const StreamSolver *s) { return s->blocks; }

void stream_admit(StreamSolver *s, const std::vector<uint32_t> &blocks, const std::vector<uint32_t> &srcv) {
    wr_graph *g = s->g;
    SegWork &w = stream_work(s);
    w.state_clean = false;
    const TileSet &ts = *g->tiles;
    const SegState &ss = w.ss;
    hipStream_t st = g->ctx->stream;
    ensure_overlay_tables(g);   // the epoch may have moved since the last admission
    const uint32_t nb = static_cast<uint32_t>(blocks.size());
    if (!nb) return;
    std::vector<uint32_t> sp(static_cast<size_t>(nb) * 64), stl(static_cast<size_t>(nb) * 64);
    for (size_t k = 0; k < sp.size(); ++k) {
        const uint32_t v = srcv[k];
        sp[k] = v == NONE ? NONE : ts.pos_of[v];
        stl[k] = v == NONE ? NONE : ts.tile_of[v];
    }
    for (uint32_t i = 0; i < nb; ++i) {
        const uint32_t b = blocks[i];
        WR_HIP(hipMemcpyAsync(w.buf.src_pos.p + static_cast<size_t>(b) * 64, sp.data() + static_cast<size_t>(i) * 64,
                              256, hipMemcpyHostToDevice, st));
        WR_HIP(hipMemcpyAsync(w.buf.src_tile.p + static_cast<size_t>(b) * 64, stl.data() + static_cast<size_t>(i) * 64,
                              256, hipMemcpyHostToDevice, st));
        launch_fill_u32(w.buf.xval.p + static_cast<size_t>(b) * std::max(ts.NB, 1u) * 64,
                        static_cast<size_t>(std::max(ts.NB, 1u)) * 64, INF, st);
        launch_fill_u8(w.buf.visited.p + static_cast<size_t>(b) * ts.T, ts.T, 0u, st);
        launch_fill_u32(w.buf.stamps.p + static_cast<size_t>(b) * ts.T, ts.T, 0u, st);
    }
    // first pass of the new rows: each source stores its in-tile distances to
    // its tile's exits as its row's exit values and flags the tiles they lead to
    std::vector<uint32_t> slots;
    for (uint32_t i = 0; i < nb; ++i)
        for (uint32_t l = 0; l < 64; ++l)
            if (srcv[static_cast<size_t>(i) * 64 + l] != NONE) slots.push_back(blocks[i] * 64 + l);
    DBuf<uint32_t> d_slots;
    upload(d_slots, g->ctx, slots, st);
    launch_ovl_seed_push(ts, ss, d_slots.p, static_cast<uint32_t>(slots.size()), st);
    WR_HIP(hipStreamSynchronize(st));
}

void stream_step(StreamSolver *s, std::vector<uint32_t> &pending) {
    wr_graph *g = s->g;
    SegWork &w = stream_work(s);
    hipStream_t st = g->ctx->stream;
    WR_HIP(hipGraphLaunch(w.exec, st));
    pending.resize(s->blocks);
    WR_HIP(hipMemcpyAsync(pending.data(), w.buf.pending.p, static_cast<size_t>(s->blocks) * 4,
                          hipMemcpyDeviceToHost, st));
    WR_HIP(hipStreamSynchronize(st));
}

void stream_gather(StreamSolver *s, const std::vector<uint32_t> &off, const std::vector<uint32_t> &picks,
                   const std::vector<uint32_t> &slot_of_pick, uint32_t *host_out) {
    wr_graph *g = s->g;
    SegWork &w = stream_work(s);
    wr_context *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = static_cast<uint32_t>(off.size()) - 1;
    std::vector<uint64_t> base(n);
    uint64_t total = 0;
    for (uint32_t o = 0; o < n; ++o) {
        base[o] = total;
        total += static_cast<uint64_t>(off[o + 1] - off[o]) * (off[o + 1] - off[o]);
    }
    if (!total) return;
    DBuf<uint32_t> d_off, d_picks, d_slot, d_out;
    DBuf<uint64_t> d_base;
    upload(d_off, ctx, off, st);
    upload(d_picks, ctx, picks, st);
    upload(d_slot, ctx, slot_of_pick, st);
    upload(d_base, ctx, base, st);
    d_out.alloc(ctx, total);
    launch_gather_ovl(n, d_off.p, d_picks.p, d_base.p, d_slot.p, 0u, s->blocks * 64u, *g->tiles, w.ss,
                      g->tiles->d_F.p, d_out.p, st);
    launch_intile_fix(ctx, *g->tiles, intile_pairs(*g->tiles, n, off.data(), picks.data(), base.data(),
                                                   [](uint32_t) { return true; }),
                      false, g->V, d_out.p, st);
    WR_HIP(hipMemcpyAsync(host_out, d_out.p, total * 4, hipMemcpyDeviceToHost, st));
    WR_HIP(hipStreamSynchronize(st));
}

namespace {
}  // namespace
}  // namespace wr

using namespace wr;

extern "C" {

wr_status wr_sssp(wr_graph *g, uint32_t S, const uint32_t *sources, uint32_t *dist, int32_t *pred,
                  uint32_t flags, void *stream) {
    WR_API_BEGIN
    const double t0 = now_ms();
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    if (S == 0) return WR_OK;
    if (!sources || !dist) fail(WR_E_INVALID, "sources or dist is NULL");
    std::vector<uint32_t> h_src;
    if (flags & WR_DEVICE_INDEX) {
        WR_HIP(hipSetDevice(g->ctx->device));
        h_src = fetch_index(sources, S, stream);
        sources = h_src.data();
    }
    if (flags & WR_PRUNE_TO_PICKS) fail(WR_E_INVALID, "WR_PRUNE_TO_PICKS applies to wr_order_matrices only");
    for (uint32_t i = 0; i < S; ++i)
        if (sources[i] >= g->V) fail(WR_E_INVALID, "source out of range");
    if (pred && g->zero_w) fail(WR_E_UNSUPPORTED, "predecessors need every weight >= 1");
    const uint32_t algo = resolve_algo(g, flags);
    const bool dev = (flags & WR_DEVICE_PTRS) != 0;
    const bool timed = (flags & WR_TIME_KERNELS) != 0;
    // events around individual kernels are recorded on the stream, so timed
    // calls launch their passes eagerly instead of replaying a graph
    const bool graph_mode = (flags & WR_NO_GRAPH_CAPTURE) == 0 && !timed;
    wr_context *ctx = g->ctx;
    WR_HIP(hipSetDevice(ctx->device));
    StreamJoin join(ctx, dev, stream);
    hipStream_t st = ctx->stream;
    const uint32_t V = g->V;
    wr_run_info info{};
    info.algo = algo;

    if (algo == WR_ALGO_EDGE_B1 || algo == WR_ALGO_EDGE_B0) {
        DBuf<uint32_t> rows, dsrc;
        uint32_t *d_rows = dist;
        if (!dev) {
            rows.alloc(ctx, static_cast<size_t>(S) * V);
            d_rows = rows.p;
        }
        dsrc.alloc(ctx, S);
        WR_HIP(hipMemcpyAsync(dsrc.p, sources, S * 4ull, hipMemcpyHostToDevice, st));
        edge_solve(g, dsrc.p, S, d_rows, algo == WR_ALGO_EDGE_B0, info);
        info.unique_sources = S;
        info.chunks = 1;
        if (pred) {
            DBuf<int32_t> dpred;
            int32_t *pp = pred;
            if (!dev) {
                dpred.alloc(ctx, static_cast<size_t>(S) * V);
                pp = dpred.p;
            }
            DBuf<uint32_t> orow;
            std::vector<uint32_t> iota(S);
            std::iota(iota.begin(), iota.end(), 0u);
            upload(orow, ctx, iota, st);
            launch_pred_rows(d_rows, S, V, dsrc.p, g->d_in_ptr.p, g->d_in_src.p, g->d_in_w.p,
                             orow.p, orow.p, pp, st);
            if (!dev)
                WR_HIP(hipMemcpyAsync(pred, pp, static_cast<size_t>(S) * V * 4, hipMemcpyDeviceToHost, st));
        }
        if (!dev) WR_HIP(hipMemcpyAsync(dist, d_rows, static_cast<size_t>(S) * V * 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipStreamSynchronize(st));
        info.total_ms = now_ms() - t0;
        g->last = info;
        return WR_OK;
    }

    Plan plan = make_plan(g, sources, S, true);
    const uint32_t U = static_cast<uint32_t>(plan.usrc.size());
    info.unique_sources = U;
    const uint32_t chunk = chunk_sources(g, algo, U, graph_mode, timed);
    // rows of each chunk (output rows whose unique source falls in it)
    std::vector<std::vector<uint32_t>> rows_of(( U + chunk - 1) / chunk);
    for (uint32_t i = 0; i < S; ++i) rows_of[plan.uidx[i] / chunk].push_back(i);
    for (uint32_t lo = 0, c = 0; lo < U; lo += chunk, ++c) {
        const uint32_t n = std::min(chunk, U - lo);
        solve_chunk(g, algo, plan.usrc, lo, n, graph_mode, info);
        info.chunks += 1;
        const auto &rows = rows_of[c];
        const uint32_t R = static_cast<uint32_t>(rows.size());
        std::vector<uint32_t> ridx(R), rvert(R), orow(R);
        for (uint32_t r = 0; r < R; ++r) {
            ridx[r] = plan.uidx[rows[r]] - lo;
            rvert[r] = sources[rows[r]];
            orow[r] = dev ? rows[r] : r;
        }
        DBuf<uint32_t> d_ridx, d_rvert, d_orow, tmp;
        upload(d_ridx, ctx, ridx, st);
        upload(d_rvert, ctx, rvert, st);
        upload(d_orow, ctx, orow, st);
        uint32_t *out = dist;
        if (!dev) {
            tmp.alloc(ctx, static_cast<size_t>(R) * V);
            out = tmp.p;
        }
        emit_rows(g, algo, R, d_ridx.p, d_rvert.p, d_orow.p, out, ridx, rvert, orow);
        if (pred) {
            DBuf<int32_t> ptmp;
            int32_t *pp = pred;
            if (!dev) {
                ptmp.alloc(ctx, static_cast<size_t>(R) * V);
                pp = ptmp.p;
            }
            launch_pred_rows(out, R, V, d_rvert.p, g->d_in_ptr.p, g->d_in_src.p, g->d_in_w.p,
                             d_orow.p, d_orow.p, pp, st);
            if (!dev) {
                std::vector<int32_t> h(static_cast<size_t>(R) * V);
                WR_HIP(hipMemcpyAsync(h.data(), pp, h.size() * 4, hipMemcpyDeviceToHost, st));
                WR_HIP(hipStreamSynchronize(st));
                for (uint32_t r = 0; r < R; ++r)
                    std::memcpy(pred + static_cast<size_t>(rows[r]) * V, h.data() + static_cast<size_t>(r) * V, V * 4ull);
            }
        }
        if (!dev) {
            std::vector<uint32_t> h(static_cast<size_t>(R) * V);
            WR_HIP(hipMemcpyAsync(h.data(), out, h.size() * 4, hipMemcpyDeviceToHost, st));
            WR_HIP(hipStreamSynchronize(st));
            for (uint32_t r = 0; r < R; ++r)
                std::memcpy(dist + static_cast<size_t>(rows[r]) * V, h.data() + static_cast<size_t>(r) * V, V * 4ull);
        }
    }
    WR_HIP(hipStreamSynchronize(st));
    info.total_ms = now_ms() - t0;
    g->last = info;
    WR_API_END
}

wr_status wr_order_matrices(wr_graph *g, uint32_t num_orders, const uint32_t *pick_offsets,
                            const uint32_t *picks, uint32_t *dist_out, int32_t *pred_out,
                            uint32_t flags, void *stream) {
    WR_API_BEGIN
    const double t0 = now_ms();
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    if (num_orders == 0) return WR_OK;
    if (!pick_offsets) fail(WR_E_INVALID, "pick_offsets is NULL");
    const bool dev_index = (flags & WR_DEVICE_INDEX) != 0;
    std::vector<uint32_t> h_off, h_picks;
    if (dev_index) {
        WR_HIP(hipSetDevice(g->ctx->device));
        h_off = fetch_index(pick_offsets, static_cast<size_t>(num_orders) + 1, stream);
        pick_offsets = h_off.data();
    }
    if (pick_offsets[0] != 0) fail(WR_E_INVALID, "pick_offsets[0] must be 0");
    uint64_t total = 0;
    std::vector<uint64_t> out_base(num_orders);
    for (uint32_t o = 0; o < num_orders; ++o) {
        if (pick_offsets[o + 1] < pick_offsets[o]) fail(WR_E_INVALID, "pick_offsets must be non-decreasing");
        const uint64_t P = pick_offsets[o + 1] - pick_offsets[o];
        out_base[o] = total;
        total += P * P;
    }
    const uint32_t NPK = pick_offsets[num_orders];
    if (NPK == 0) return WR_OK;
    if (!picks || !dist_out) fail(WR_E_INVALID, "picks or dist_out is NULL");
    if (dev_index) {
        h_picks = fetch_index(picks, NPK, stream);
        picks = h_picks.data();
    }
    for (uint32_t k = 0; k < NPK; ++k)
        if (picks[k] >= g->V) fail(WR_E_INVALID, "pick out of range");
    if (pred_out && g->zero_w) fail(WR_E_UNSUPPORTED, "predecessors need every weight >= 1");
    const bool prune = (flags & WR_PRUNE_TO_PICKS) != 0;
    if (prune && pred_out) fail(WR_E_INVALID, "WR_PRUNE_TO_PICKS leaves rows beyond the picks unfinished: no pred_out");
    const uint32_t algo = resolve_algo(g, flags);
    if (prune && algo != WR_ALGO_OVERLAY) fail(WR_E_UNSUPPORTED, "WR_PRUNE_TO_PICKS runs on the overlay schedule only");
    const bool dev = (flags & WR_DEVICE_PTRS) != 0;
    const bool timed = (flags & WR_TIME_KERNELS) != 0;
    // events around individual kernels are recorded on the stream, so timed
    // calls launch their passes eagerly instead of replaying a graph
    const bool graph_mode = (flags & WR_NO_GRAPH_CAPTURE) == 0 && !timed;
    wr_context *ctx = g->ctx;
    WR_HIP(hipSetDevice(ctx->device));
    StreamJoin join(ctx, dev, stream);
    hipStream_t st = ctx->stream;
    const uint32_t V = g->V;
    wr_run_info info{};
    info.algo = algo;

    g_trace.start(t0);
    g_trace.mark("validate", now_ms());
    std::vector<uint32_t> hoff(pick_offsets, pick_offsets + num_orders + 1);
    std::vector<uint32_t> hpicks(picks, picks + NPK);
    Workspace &cws = workspace(g);
    DBuf<uint32_t> &d_off = cws.call_off, &d_picks = cws.call_picks, &d_sidx = cws.call_sidx;
    DBuf<uint64_t> &d_base = cws.call_base;
    upload_reuse(d_off, ctx, hoff, st);
    upload_reuse(d_picks, ctx, hpicks, st);
    upload_reuse(d_base, ctx, out_base, st);
    DBuf<uint32_t> dout_tmp;
    uint32_t *dout = dist_out;
    if (!dev) {
        dout_tmp.alloc(ctx, static_cast<size_t>(total));
        dout = dout_tmp.p;
    }

    if (algo == WR_ALGO_EDGE_B1 || algo == WR_ALGO_EDGE_B0) {
        // one order at a time, its picks as the N sources
        uint32_t maxP = 0;
        for (uint32_t o = 0; o < num_orders; ++o) maxP = std::max(maxP, hoff[o + 1] - hoff[o]);
        DBuf<uint32_t> rows, d_local;
        rows.alloc(ctx, static_cast<size_t>(maxP) * V);
        std::vector<uint32_t> local(NPK);
        for (uint32_t o = 0; o < num_orders; ++o)
            for (uint32_t k = hoff[o]; k < hoff[o + 1]; ++k) local[k] = k - hoff[o];
        upload(d_local, ctx, local, st);
        for (uint32_t o = 0; o < num_orders; ++o) {
            const uint32_t a = hoff[o], P = hoff[o + 1] - a;
            if (!P) continue;
            edge_solve(g, d_picks.p + a, P, rows.p, algo == WR_ALGO_EDGE_B0, info);
            launch_gather_rows(1, d_off.p + o, d_picks.p, d_base.p + o, d_local.p, rows.p, V, dout, st);
            if (pred_out) {
                DBuf<int32_t> ptmp;
                int32_t *pp = pred_out + static_cast<size_t>(a) * V;
                if (!dev) {
                    ptmp.alloc(ctx, static_cast<size_t>(P) * V);
                    pp = ptmp.p;
                }
                DBuf<uint32_t> orow;
                std::vector<uint32_t> iota(P);
                std::iota(iota.begin(), iota.end(), 0u);
                upload(orow, ctx, iota, st);
                launch_pred_rows(rows.p, P, V, d_picks.p + a, g->d_in_ptr.p, g->d_in_src.p,
                                 g->d_in_w.p, orow.p, orow.p, pp, st);
                if (!dev)
                    WR_HIP(hipMemcpyAsync(pred_out + static_cast<size_t>(a) * V, pp,
                                          static_cast<size_t>(P) * V * 4, hipMemcpyDeviceToHost, st));
            }
        }
        info.unique_sources = NPK;
        info.chunks = num_orders;
    } else {
        g_trace.mark("uploads", now_ms());
        Plan plan = make_plan(g, picks, NPK, true);
        g_trace.mark("plan", now_ms());
        const uint32_t U = static_cast<uint32_t>(plan.usrc.size());
        info.unique_sources = U;
        upload_reuse(d_sidx, ctx, plan.uidx, st);
        const uint32_t chunk = chunk_sources(g, algo, U, graph_mode, timed);
        for (uint32_t lo = 0; lo < U; lo += chunk) {
            const uint32_t n = std::min(chunk, U - lo);
            // overlay: the in-tile values of entries whose picks share a tile
            // depend only on the tiles, so they are computed on the side
            // stream while the chunk relaxes, and applied after the gather
            IntileJob &job = workspace(g).intile;
            hipEvent_t ev_side = nullptr;
            std::function<void()> overlap;
            hipEvent_t ev_ready = nullptr;
            if (algo == WR_ALGO_OVERLAY) {
                // the fix-up reads only the tiles' arc tables, which are on the
                // device once the work queued on st so far is done
                WR_HIP(hipEventCreateWithFlags(&ev_ready, hipEventDisableTiming));
                WR_HIP(hipEventRecord(ev_ready, st));
                // runs once the first passes are queued, so the host builds the
                // pair list while the GPU relaxes; the side stream starts once
                // the heavy first passes are done (the mid-batch event), as the
                // fix-up depends only on the tile tables
                overlap = [&]() {
                    const IntileWork iw = intile_pairs(*g->tiles, num_orders, pick_offsets, picks, out_base.data(),
                                                       [&](uint32_t k) { return plan.uidx[k] >= lo && plan.uidx[k] < lo + n; });
                    Workspace &ows = workspace(g);
                    WR_HIP(hipStreamWaitEvent(ctx->side, ows.mid_valid ? ows.ev_mid : ev_ready, 0));
                    job.upload_and_launch(ctx, *g->tiles, iw, false, g->V, nullptr, ctx->side);
                    WR_HIP(hipEventCreateWithFlags(&ev_side, hipEventDisableTiming));
                    WR_HIP(hipEventRecord(ev_side, ctx->side));
                    g_trace.mark("intile_setup", now_ms());
                };
            }
            std::function<void()> refine;
            if (prune)
                refine = [&]() {
                    SegWork &sw = *workspace(g).seg;
                    launch_bound_refine(num_orders, d_off.p, d_picks.p, d_sidx.p, lo, n, *g->tiles, sw.ss,
                                        g->tiles->d_F.p, sw.bound.p, sw.bound_tmp.p, st);
                };
            solve_chunk(g, algo, plan.usrc, lo, n, graph_mode, info, overlap, refine);
            g_trace.mark("solve", now_ms());
            info.chunks += 1;
            if (algo == WR_ALGO_OVERLAY) {
                launch_gather_ovl(num_orders, d_off.p, d_picks.p, d_base.p, d_sidx.p, lo, n, *g->tiles,
                                  workspace(g).seg->ss, g->tiles->d_F.p, dout, st);
                WR_HIP(hipStreamWaitEvent(st, ev_side, 0));
                (void)hipEventDestroy(ev_side);
                (void)hipEventDestroy(ev_ready);
                job.apply(dout, st);
            }
            else if (algo == WR_ALGO_SEGMENTED)
                launch_gather_seg(num_orders, d_off.p, d_picks.p, d_base.p, d_sidx.p, lo, n, *g->tiles,
                                  workspace(g).seg->ss, dout, st);
            else
                launch_gather_blk(num_orders, d_off.p, d_picks.p, d_base.p, d_sidx.p, lo, n,
                                  workspace(g).blk->dist.p, V, dout, st);
            if (pred_out) {
                // predecessor rows of the picks whose source is in this chunk,
                // a bounded group of rows at a time
                std::vector<uint32_t> ks;
                for (uint32_t k = 0; k < NPK; ++k)
                    if (plan.uidx[k] >= lo && plan.uidx[k] < lo + n) ks.push_back(k);
                const uint32_t RG = 64;
                DBuf<uint32_t> rtmp;
                rtmp.alloc(ctx, static_cast<size_t>(std::min<size_t>(RG, ks.size())) * V);
                DBuf<int32_t> ptmp;
                if (!dev) ptmp.alloc(ctx, static_cast<size_t>(std::min<size_t>(RG, ks.size())) * V);
                for (size_t g0 = 0; g0 < ks.size(); g0 += RG) {
                    const uint32_t R = static_cast<uint32_t>(std::min<size_t>(RG, ks.size() - g0));
                    std::vector<uint32_t> ridx(R), rvert(R), orow(R), prow(R);
                    for (uint32_t r = 0; r < R; ++r) {
                        const uint32_t k = ks[g0 + r];
                        ridx[r] = plan.uidx[k] - lo;
                        rvert[r] = picks[k];
                        orow[r] = r;
                        prow[r] = dev ? k : r;
                    }
                    DBuf<uint32_t> d_ridx, d_rvert, d_orow, d_prow;
                    upload(d_ridx, ctx, ridx, st);
                    upload(d_rvert, ctx, rvert, st);
                    upload(d_orow, ctx, orow, st);
                    upload(d_prow, ctx, prow, st);
                    emit_rows(g, algo, R, d_ridx.p, d_rvert.p, d_orow.p, rtmp.p, ridx, rvert, orow);
                    int32_t *pp = dev ? pred_out : ptmp.p;
                    launch_pred_rows(rtmp.p, R, V, d_rvert.p, g->d_in_ptr.p, g->d_in_src.p,
                                     g->d_in_w.p, d_orow.p, d_prow.p, pp, st);
                    if (!dev) {
                        std::vector<int32_t> h(static_cast<size_t>(R) * V);
                        WR_HIP(hipMemcpyAsync(h.data(), ptmp.p, h.size() * 4, hipMemcpyDeviceToHost, st));
                        WR_HIP(hipStreamSynchronize(st));
                        for (uint32_t r = 0; r < R; ++r)
                            std::memcpy(pred_out + static_cast<size_t>(ks[g0 + r]) * V,
                                        h.data() + static_cast<size_t>(r) * V, V * 4ull);
                    }
                }
                WR_HIP(hipStreamSynchronize(st));
            }
        }
    }
    g_trace.mark("gather", now_ms());
    if (!dev) WR_HIP(hipMemcpyAsync(dist_out, dout, static_cast<size_t>(total) * 4, hipMemcpyDeviceToHost, st));
    SegWork *sw = workspace(g).seg.get();
    if (algo == WR_ALGO_OVERLAY && sw && sw->overlay && !sw->state_clean) {
        // the results are complete at ev_done; the exit values of the rows
        // this call used are reset behind it, while the host moves on
        Workspace &ws = workspace(g);
        if (!ws.ev_done) WR_HIP(hipEventCreateWithFlags(&ws.ev_done, hipEventDisableTiming));
        WR_HIP(hipEventRecord(ws.ev_done, st));
        launch_fill_u32(sw->buf.xval.p, static_cast<size_t>(sw->dirty_rows) * std::max(g->tiles->NB, 1u) * 64,
                        INF, st);
        sw->state_clean = true;
        WR_HIP(hipEventSynchronize(ws.ev_done));
    } else {
        WR_HIP(hipStreamSynchronize(st));
    }
    info.total_ms = now_ms() - t0;
    g_trace.mark("sync", now_ms());
    g_trace.flush("order_matrices");
    g->last = info;
    WR_API_END
}

wr_status wr_graph_last_run(const wr_graph *g, wr_run_info *info) {
    WR_API_BEGIN
    if (!g || !info) fail(WR_E_INVALID, "NULL argument");
    *info = g->last;
    WR_API_END
}

wr_status wr_graph_set_schedule(wr_graph *g, uint32_t tile_vertices, uint32_t waves_per_group,
                                uint32_t passes_per_replay) {
    WR_API_BEGIN
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    uint32_t t = tile_vertices ? tile_vertices : g->tile_vertices;
    uint32_t wv = waves_per_group ? waves_per_group : g->waves_per_group;
    // tile sizes up to 512 run the source-blocked kernel (64 sources per
    // workgroup item); larger tiles run one source per wave
    const uint32_t lanes = t <= 512 ? 64u : 1u;
    const bool ok = lanes == 64 ? ((t == 256 || t == 512) && (wv == 8 || wv == 16))
                                : ((t == 1024 && (wv == 4 || wv == 8)) || (t == 2048 && (wv == 4 || wv == 8)) ||
                                   (t == 4096 && wv == 2));
    if (!ok) fail(WR_E_INVALID, "unsupported (tile_vertices, waves_per_group) pair");
    g->tile_vertices = t;
    g->waves_per_group = wv;
    g->lanes = lanes;
    if (passes_per_replay) g->passes_per_replay = std::max(2u, passes_per_replay & ~1u);
    destroy_workspace(g->ws);
    g->ws = nullptr;
    WR_API_END
}

}  // extern "C"
