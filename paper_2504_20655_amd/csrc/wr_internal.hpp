// Internal declarations of the routing library: device buffers, graph and
// tile tables, work plans and the kernel launchers implemented in
// kernels.hip.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wroute.h"

namespace wr {

constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr uint32_t LANES = 64;            // CDNA wavefront width; also S_b of the blocked layout

// ---------------------------------------------------------------- errors
struct Error {
    wr_status st;
    std::string msg;
};
[[noreturn]] void fail(wr_status st, const std::string &msg);
void set_last_error(const std::string &msg);
void clear_last_error();

#define WR_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            ::wr::fail(WR_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Fault injection for host-forced failure tests: WR_FAULT="alloc:N" fails the
// N-th device allocation, "launch:N" the N-th kernel launch (1-based, counted
// per process).
bool fault_alloc_now();
bool fault_launch_now();
void check_launch(const char *what);

}  // namespace wr

// Every ABI entry point runs its body between these: errors thrown as
// wr::Error become the returned status plus the thread-local message.
#define WR_API_BEGIN try { ::wr::clear_last_error();
#define WR_API_END                                         \
    return WR_OK;                                          \
    }                                                      \
    catch (const ::wr::Error &e) {                         \
        ::wr::set_last_error(e.msg);                       \
        return e.st;                                       \
    }                                                      \
    catch (const std::bad_alloc &) {                       \
        ::wr::set_last_error("host allocation failed");    \
        return WR_E_NOMEM;                                 \
    }                                                      \
    catch (...) {                                          \
        ::wr::set_last_error("unexpected exception");      \
        return WR_E_INTERNAL;                              \
    }

// ----------------------------------------------------------------- context
struct wr_context {
    int device = 0;
    int num_cus = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    hipStream_t stream = nullptr;   // internal stream for host-pointer calls
    hipStream_t side = nullptr;     // second internal stream (work that overlaps the relaxation)

    void *alloc(size_t bytes);      // throws WR_E_NOMEM / WR_E_DEVICE
    void release(void *p, size_t bytes);
    uint64_t available() const { return used.load() >= budget ? 0 : budget - used.load(); }
};

namespace wr {

// Device buffer owned by a context; freed on destruction.
template <class T>
struct DBuf {
    wr_context *ctx = nullptr;
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept { *this = std::move(o); }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            reset();
            ctx = o.ctx; p = o.p; n = o.n;
            o.ctx = nullptr; o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DBuf() { reset(); }
    void alloc(wr_context *c, size_t count) {
        reset();
        ctx = c;
        n = count;
        p = count ? static_cast<T *>(c->alloc(count * sizeof(T))) : nullptr;
    }
    void reset() {
        if (p && ctx) ctx->release(p, n * sizeof(T));
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

template <class T>
void upload(DBuf<T> &d, wr_context *ctx, const std::vector<T> &h, hipStream_t st) {
    d.alloc(ctx, h.size());
    if (!h.empty()) WR_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// Grow-only buffers for per-call arrays: reallocated only when too small, so
// repeated calls do not allocate (the caller orders reuse on its stream).
template <class T>
void reserve(DBuf<T> &d, wr_context *ctx, size_t count) {
    if (d.n >= count && d.p) return;
    d.alloc(ctx, std::max<size_t>(count, d.n * 2));
}
template <class T>
void upload_reuse(DBuf<T> &d, wr_context *ctx, const std::vector<T> &h, hipStream_t st) {
    reserve(d, ctx, std::max<size_t>(h.size(), 1));
    if (!h.empty()) WR_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// ---------------------------------------------------------- LDS tile tables
// A segmentation turned into LDS tiles.  Tiled vertices (those incident to at
// least one arc) are renumbered tile by tile into "positions" 0..Vt-1;
// position = tile_base[t] + local index, local index < tile size.
struct TileSet {
    uint32_t num_segments = 0;
    uint32_t T = 0;               // tiles
    uint32_t Vt = 0;              // tiled vertices
    uint32_t NP = 0;              // ports: boundary-in vertices (an arc from another tile ends there)
    uint32_t NB = 0;              // boundary-out vertices (an arc to another tile starts there)
    uint32_t tile_cap = 0;        // maximum tile size the tables were built for
    uint64_t cross_arcs = 0;
    uint32_t max_ports = 0;       // most ports of one tile
    uint32_t max_exits = 0;       // most boundary-out vertices of one tile
    uint32_t max_cross = 0;       // most cross-tile arcs leaving one tile
    uint32_t max_cross_in = 0;    // most cross-tile arcs entering one tile
    // overlay boundary tables F[pos][64] (lane i = port i of the tile) and the
    // weight epoch they were computed for
    DBuf<uint32_t> d_F;
    uint64_t custom_epoch = ~0ull;
    // overlay pass staging.  Per tile a header {first port, first exit, first
    // cross arc, ports | exits << 8 | cross arcs << 16}; per tile t, X_t + 1
    // entries from bo_base[t] + t: each exit's first cross arc relative to
    // the tile's; and the exits' table rows packed [NB][ovl_em] (entries
    // beyond the tile's ports INF) for the epoch of d_F.
    uint32_t ovl_em = 0;
    std::vector<uint32_t> ovl_hdr, bo_xbeg;
    // per tile, the key sources are ordered by (see tile_order_keys), and
    // the tile's rank in (key, tile) order
    std::vector<uint64_t> order_key;
    std::vector<uint32_t> order_rank;
    DBuf<uint32_t> d_ovl_hdr, d_bo_xbeg, d_Fx;
    // pull form of the overlay: per port p its incoming cross arcs
    // k in [pin_off[p], pin_off[p + 1]): the arc's index in the x_ arrays
    // (pin_xa), its source exit (pin_exit, an index of the exit tables) and
    // the port's index in its tile (pin_lport); for the epoch of d_F the
    // packed records d_pin_rec[k] = {source exit, w | local port << 16}; per
    // tile {first incoming arc, incoming arcs} (ovl_hdr2)
    std::vector<uint32_t> pin_off, pin_xa, pin_exit, pin_lport, ovl_hdr2;
    DBuf<uint32_t> d_pin_off, d_pin_xa, d_pin_exit, d_pin_lport, d_ovl_hdr2;
    DBuf<uint2> d_pin_rec;
    // exit tables B[pos][64] of the epoch of d_F (lane j: in-tile distance to
    // exit j of the tile), and positions' vertices on the device
    DBuf<uint32_t> d_B, d_vert_of;

    // host copies
    std::vector<uint32_t> tile_of;      // [V]  tile or NONE
    std::vector<uint32_t> pos_of;       // [V]  position or NONE
    std::vector<uint32_t> vert_of;      // [Vt] vertex of a position
    std::vector<uint32_t> tile_base;    // [T+1]
    std::vector<uint32_t> l_off;        // [Vt+1] in-tile out-arc offsets
    std::vector<uint32_t> l_arc;        // packed (local dst << 16) | w   (w < 65536)
    std::vector<uint32_t> x_off;        // [Vt+1] cross-tile out-arc offsets
    std::vector<uint32_t> x_port;       // target port
    std::vector<uint32_t> x_w;          // weight
    std::vector<uint32_t> x_tile;       // target tile
    std::vector<uint32_t> port_base;    // [T+1]
    std::vector<uint32_t> port_local;   // local index of each port in its tile
    std::vector<uint32_t> bo_base;      // [T+1]
    std::vector<uint32_t> bo_local;     // local index of each boundary-out vertex
    std::vector<uint32_t> arc_slot;     // [E] where CSR arc e lives: l_arc index, or 0x80000000|x index
    std::vector<uint32_t> li_off;       // [Vt+1] in-tile in-arc offsets (pull form)
    std::vector<uint32_t> li_arc;       // packed (local src << 16) | w
    std::vector<uint32_t> arc_slot_in;  // [E] li_arc index of an in-tile arc, NONE for cross arcs

    // device copies
    DBuf<uint32_t> d_tile_of, d_pos_of, d_tile_base, d_l_off, d_l_arc, d_x_off, d_x_port, d_x_w,
        d_x_tile, d_port_base, d_port_local, d_bo_base, d_bo_local, d_arc_slot, d_li_off, d_li_arc,
        d_arc_slot_in;
};

}  // namespace wr

namespace wr {
struct Workspace;
void destroy_workspace(Workspace *ws);
}  // namespace wr

// ------------------------------------------------------------------- graph
struct wr_graph {
    wr_context *ctx = nullptr;
    uint32_t V = 0, E = 0;
    uint32_t n_incident = 0;   // vertices incident to an arc (overflow bound)
    std::vector<uint32_t> row_ptr, col, w;   // host mirror at the current epoch
    std::vector<uint32_t> in_pos_of_arc;     // [E] position of arc e in the in-CSR
    uint64_t epoch = 0;
    uint32_t max_w = 0;
    uint64_t zero_w = 0;       // number of arcs with weight 0

    wr::DBuf<uint32_t> d_row_ptr, d_col, d_w;          // out-CSR
    wr::DBuf<uint32_t> d_in_ptr, d_in_src, d_in_w;     // in-CSR (pull)
    wr::DBuf<uint32_t> d_in_pos_of_arc;
    wr::DBuf<uint32_t> d_arc_src;                      // [E] tail of each arc (edge-list baseline), lazy

    wr::TileSet *tiles = nullptr;
    uint64_t tiles_gen = 0;            // bumped whenever `tiles` is rebuilt
    wr::Workspace *ws = nullptr;       // cached per-call work buffers and captured graphs
    bool tiles_user = false;           // segmentation given by the caller
    std::vector<uint32_t> user_seg;    // caller's segment map (rebuilt on tile-size change)
    uint32_t user_num_segments = 0;
    uint32_t grid_W = 0, grid_H = 0, grid_L = 0, grid_tw = 0, grid_th = 0;   // last segment_grid spec

    // schedule
    uint32_t tile_vertices = 256;
    uint32_t waves_per_group = 8;
    uint32_t lanes = 64;               // 64: source-blocked segment kernel; 1: one source per wave
    uint32_t sources_per_unit = 0;     // 0 = 4 * waves_per_group
    uint32_t passes_per_replay = 8;

    wr_run_info last{};
    ~wr_graph();
};

namespace wr {

// -------------------------------------------------------- kernel launchers
// (kernels.hip)  All enqueue on `st`.
void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
void launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t st);

// blocked layout dist[b][v][64]: source 64*b + l of a chunk at vertex v
void launch_blk_seed(uint32_t *dist, uint32_t V, uint32_t S, const uint32_t *src, hipStream_t st);
void launch_sweep_pull(uint32_t *dist, uint32_t V, uint32_t nb, const uint32_t *in_ptr,
                       const uint32_t *in_src, const uint32_t *in_w, uint32_t *changed,
                       uint32_t grid, hipStream_t st);
// frontier items are (block << 32 | vertex); stamps[b*V+v] = pass stamp when queued
void launch_frontier_seed(uint64_t *list, uint32_t *count, uint32_t S, const uint32_t *src,
                          uint32_t V, hipStream_t st);
void launch_frontier_push(uint32_t *dist, uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                          const uint32_t *w, const uint64_t *list_in, const uint32_t *count_in,
                          uint64_t *list_out, uint32_t *count_out, uint32_t *stamps,
                          const uint32_t *pass_ctr, uint32_t grid, hipStream_t st);
// zero count_next, add count_cur into stats[0], (count_cur > 0) into stats[1], ++pass_ctr
void launch_pass_prologue(uint32_t *count_next, const uint32_t *count_cur,
                          unsigned long long *stats, uint32_t *pass_ctr, hipStream_t st);
// row r of the chunk state (source row_src_idx[r]) goes to out + out_row[r]*V
void launch_blk_emit(const uint32_t *dist, uint32_t V, uint32_t rows, const uint32_t *row_src_idx,
                     const uint32_t *out_row, uint32_t *out, hipStream_t st);

// segmented schedule: device state of one chunk of S sources
struct SegState {
    uint32_t S = 0;
    uint32_t *gdist = nullptr;      // [S][Vt]
    uint32_t *inbox = nullptr;      // [S][NP]
    uint32_t *xval = nullptr;       // [S][NB][64] exit values (overlay schedule)
    uint8_t *visited = nullptr;     // [S][T]
    uint32_t *stamps = nullptr;     // [S][T]
    uint32_t *cnt = nullptr;        // [2][T]
    uint32_t *bucket = nullptr;     // [2][T][S]
    uint32_t *tiles = nullptr;      // [2][T]
    uint32_t *ntiles = nullptr;     // [2]
    uint2 *units = nullptr;         // [max units]
    uint32_t *nunits = nullptr;     // [1]; the overlay steps use nunits[3] for parity 1
    uint32_t *cursor = nullptr;     // [1]; the overlay steps use cursor[3] for parity 1
    uint32_t *pass_ctr = nullptr;   // [1]
    unsigned long long *stats = nullptr;   // [2]: items, passes with work
    const uint32_t *src_pos = nullptr;     // [sources] position or NONE
    const uint32_t *src_tile = nullptr;    // [sources] tile or NONE
    uint32_t lanes_log2 = 0;   // 0: a state row per source; 6: per block of 64 sources
    uint32_t nsrc = 0;         // sources of the chunk (blocked layout: lanes beyond are idle)
    uint8_t *flags = nullptr;  // [T][S] activation flags (overlay schedule), else null
    uint32_t *pending = nullptr;   // [S] blocks with set flags after a replay (overlay schedule)
    uint32_t *tile_visits = nullptr;   // [T] overlay visits of each tile (work counter)
    uint32_t *wave_stores = nullptr;   // [wave slots] exit values each pass wave stored (work counter)
};
// activates (s, tile of source s) for the chunk's sources s < n
void launch_seg_seed_n(const TileSet &ts, const SegState &ss, uint32_t n, hipStream_t st);
// one pass: prologue (zero next counters) + plan (units) + relaxation
// ev (optional): events recorded right before / after the relaxation kernel
void launch_seg_step(const TileSet &ts, const SegState &ss, uint32_t parity, uint32_t tile_cap,
                     uint32_t waves, uint32_t G, uint32_t grid, hipStream_t st,
                     hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);
uint32_t seg_pass_lds_bytes(uint32_t tile_cap, uint32_t waves, uint32_t lanes);
void launch_seg_emit(const TileSet &ts, const SegState &ss, uint32_t V, uint32_t rows,
                     const uint32_t *row_src_idx, const uint32_t *row_src_vertex,
                     const uint32_t *out_row, uint32_t *out, hipStream_t st);

// Device buffers of one segmented state of S_cap state rows (sources, or
// blocks of 64 sources with lanes = 64; see SegState).
struct SegBuffers {
    uint32_t S_cap = 0, G = 0, lanes = 1;
    DBuf<uint32_t> gdist, inbox, xval, stamps, cnt, bucket, tiles, ctr, src_pos, src_tile, pending;
    DBuf<uint32_t> tile_visits, wave_stores;
    uint32_t wave_slots = 0;   // workgroups x waves of the widest overlay pass launch
    DBuf<uint8_t> visited, flags;
    DBuf<uint2> units;
    DBuf<unsigned long long> stats;
    SegState ss;
    // with_flags: activation by flags [T][S_cap] (overlay schedule)
    void init(wr_context *ctx, const TileSet &ts, uint32_t S_cap, uint32_t G, uint32_t lanes, bool with_flags);
    // device bytes per state row
    static uint64_t bytes_per_row(const TileSet &ts, uint32_t G, uint32_t lanes, bool overlay);
};
// Streaming overlay state for continuous batching: a fixed set of block rows
// (64 source lanes each) that are seeded, relaxed and read out independently,
// so new sources join between replays while older ones are still relaxing.
struct StreamSolver;
// Throws WR_E_UNSUPPORTED when the graph's tiling cannot run the overlay
// schedule; `blocks` is the number of rows wanted (bounded by the budget).
StreamSolver *stream_create(wr_graph *g, uint32_t blocks);
void stream_destroy(StreamSolver *s);
uint32_t stream_blocks(const StreamSolver *s);
// Bytes of device state per block row of the streaming schedule.
uint64_t stream_bytes_per_block(wr_graph *g);
// Resets the listed rows and seeds them with srcv[i * 64 + lane] (NONE for
// an empty lane), then runs their first pass (the sources' own tiles).
void stream_admit(StreamSolver *s, const std::vector<uint32_t> &blocks, const std::vector<uint32_t> &srcv);
// One replay of passes over every row; pending[b] != 0 while row b has work.
void stream_step(StreamSolver *s, std::vector<uint32_t> &pending);
// Order matrices of converged rows into host memory: picks of order o are
// picks[off[o] .. off[o+1]) with source slot (row * 64 + lane) slot_of_pick.
void stream_gather(StreamSolver *s, const std::vector<uint32_t> &off, const std::vector<uint32_t> &picks,
                   const std::vector<uint32_t> &slot_of_pick, uint32_t *host_out);

// Persistent grid size of the pass kernel for this schedule.
uint32_t seg_pass_grid(const wr_context *ctx, uint32_t tile_cap, uint32_t waves, uint32_t lanes);
// Captures K passes (parities 0,1,0,...) into an instantiated graph.
hipGraphExec_t capture_seg_passes(const TileSet &ts, const SegState &ss, uint32_t K, uint32_t tile_cap,
                                  uint32_t waves, uint32_t G, uint32_t grid, hipStream_t st);

// overlay schedule: per-epoch boundary tables F[pos][port] of every tile,
// dense min-plus passes over (tile, block) items, and the read-outs
// reverse = false: F (from ports); reverse = true: B[pos][j] = in-tile
// distance from pos to exit j of its tile
void launch_ovl_custom(const TileSet &ts, uint32_t tile_cap, uint32_t *F, uint32_t grid, hipStream_t st,
                       bool reverse);
// first overlay pass: stores each source slot's in-tile distances to its
// tile's exits (B rows) as the exit values of its block and flags the tiles
// the exits lead to; slots == NULL means the slots 0 .. nslots-1
void launch_ovl_seed_push(const TileSet &ts, const SegState &ss, const uint32_t *slots, uint32_t nslots,
                          hipStream_t st);
// In-tile fix-ups after an overlay read-out: groups of up to 64 sources of one
// tile (4 words per group: tile, lanes, first pair, end pair; 64 source local
// indices per group).  Pair mode: pair_key = lane << 16 | target local index,
// pair_out = output index.  Full mode: row = output row per lane, every tile
// vertex written.  out[...] becomes min(out[...], in-tile distance).
struct IntileWork {
    std::vector<uint32_t> grp, src_local, row, pair_key;
    std::vector<uint64_t> pair_out;
};
void launch_intile_fix(wr_context *ctx, const TileSet &ts, const IntileWork &w, bool full, uint32_t V,
                       uint32_t *out, hipStream_t st);
// The pairs form split in two, so it can run beside the relaxation: launch
// with out == NULL computes the in-tile values into a device buffer (its
// inputs live as long as the job, whose buffers are reused by later jobs);
// apply() lowers out[...] by them.
struct IntileJob {
    uint32_t ng = 0, npairs = 0;
    DBuf<uint32_t> d_grp, d_src, d_row, d_key, d_val;
    DBuf<uint64_t> d_out;
    void upload_and_launch(wr_context *ctx, const TileSet &ts, const IntileWork &w, bool full, uint32_t V,
                           uint32_t *out, hipStream_t st);
    void apply(uint32_t *out, hipStream_t st) const;
};
// entries per packed table row of the overlay pass (ports rounded up to 4)
uint32_t ovl_row_entries(const TileSet &ts);
// packs the exits' rows of F into d_Fx
void launch_ovl_pack(const TileSet &ts, hipStream_t st);
// packs d_pin_rec from the current cross-arc weights
void launch_ovl_pin_rec(const TileSet &ts, hipStream_t st);
// one overlay pass: prologue + plan from the flags + the pass; count_after
// adds the number of waves that still see set flags to ntiles[parity ^ 1]
void launch_ovl_step(const TileSet &ts, const SegState &ss, uint32_t parity, uint32_t G, uint32_t grid,
                     const uint32_t *F, bool count_after, hipStream_t st, hipEvent_t ev_begin = nullptr,
                     hipEvent_t ev_end = nullptr, const uint32_t *bound = nullptr);
// target bounds of the chunk's sources (bound[s] for s < chunk_n): bound =
// min(bound, max over each source's order pairs of the current overlay
// value); tmp (chunk_n words) must be 0 and is left 0
void launch_bound_refine(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                         const uint32_t *src_idx_of_pick, uint32_t chunk_lo, uint32_t chunk_n, const TileSet &ts,
                         const SegState &ss, const uint32_t *F, uint32_t *bound, uint32_t *tmp, hipStream_t st);
// full rows: out_row[r] * V .. gets the row of the source at row_src_vertex[r];
// the rows' sources are grouped by 64-source block: group g covers block
// grp_block[g], lane l of it goes to row lane_row[g * 64 + l] (NONE: none)
void launch_ovl_emit(const TileSet &ts, const SegState &ss, const uint32_t *F, uint32_t V, uint32_t rows,
                     const uint32_t *row_src_vertex, const uint32_t *out_row, const uint32_t *grp_block,
                     const uint32_t *lane_row, uint32_t ngroups, uint32_t num_cus, uint32_t *out, hipStream_t st);
void launch_gather_ovl(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                       const uint64_t *out_base, const uint32_t *src_idx_of_pick, uint32_t chunk_lo,
                       uint32_t chunk_n, const TileSet &ts, const SegState &ss, const uint32_t *F,
                       uint32_t *out, hipStream_t st);
uint32_t ovl_pass_lds_bytes(const TileSet &ts);
uint32_t ovl_max_exits();
uint32_t ovl_max_entries();
uint32_t ovl_max_cross();
uint32_t ovl_waves();   // waves (= blocks per unit) of the overlay pass

// optimal open route per order (Held and Karp over stop subsets, one
// workgroup per order): orders of at most route_max_stops() stops; the
// matrices start at dist + mbase[o]; *overflow is raised when a partial
// length reaches WR_INF in 32 bits
uint32_t route_max_stops();
uint32_t route_lds_bytes(uint32_t nmax);
// the permutation-per-thread baseline: best[o] must start at ~0 (one 64-bit
// key per order); orders of at most route_enumerate_max_stops() stops
uint32_t route_enumerate_max_stops();
void launch_route_perm(uint32_t num_orders, const uint32_t *off, const uint64_t *mbase, const uint32_t *dist,
                       unsigned long long *best, uint64_t *len_out, uint32_t *route_out, uint32_t *overflow,
                       uint32_t nmax, hipStream_t st);
void launch_route_hk(uint32_t num_orders, const uint32_t *off, const uint64_t *mbase, const uint32_t *dist,
                     uint64_t *len_out, uint32_t *route_out, uint32_t *overflow, uint32_t nmax, uint32_t grid,
                     hipStream_t st);

// cluster-decomposed route per order (K-means on integer positions, each
// cluster's subset programme, the cheapest chaining); *err gets
// route_clustered_err_range() / _err_cluster() bits
uint32_t route_clustered_max_stops();
uint32_t route_clustered_max_clusters();
uint32_t route_clustered_lds_bytes();
void launch_route_clustered(uint32_t num_orders, const uint32_t *off, const uint64_t *mbase, const uint32_t *dist,
                            const int32_t *xy, uint32_t m, uint64_t *len_out, uint32_t *route_out, uint32_t *m_out,
                            uint32_t *err, uint32_t grid, hipStream_t st);

// order gathers: out[out_base[o] + i*P + j] = d(p_i, p_j)
void launch_gather_rows(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                        const uint64_t *out_base, const uint32_t *row_of_pick, const uint32_t *rows,
                        uint32_t V, uint32_t *out, hipStream_t st);
void launch_gather_blk(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                       const uint64_t *out_base, const uint32_t *src_idx_of_pick, uint32_t chunk_lo,
                       uint32_t chunk_n, const uint32_t *dist, uint32_t V, uint32_t *out,
                       hipStream_t st);
void launch_gather_seg(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                       const uint64_t *out_base, const uint32_t *src_idx_of_pick, uint32_t chunk_lo,
                       uint32_t chunk_n, const TileSet &ts, const SegState &ss, uint32_t *out,
                       hipStream_t st);

// canonical predecessor: row r is read at rows + in_row[r]*V and written at
// pred + out_row[r]*V
void launch_pred_rows(const uint32_t *rows, uint32_t nrows, uint32_t V, const uint32_t *row_src_vertex,
                      const uint32_t *in_ptr, const uint32_t *in_src, const uint32_t *in_w,
                      const uint32_t *in_row, const uint32_t *out_row, int32_t *pred, hipStream_t st);

// paper-structured edge-list baseline: dist[N][V] in place, one thread per arc
void launch_edge_round(const uint32_t *arc_src, const uint32_t *col, const uint32_t *w, uint32_t E,
                       uint32_t *dist, uint32_t V, uint32_t N, uint32_t *changed, hipStream_t st);
void launch_rows_seed(uint32_t *dist, uint32_t V, uint32_t N, const uint32_t *src, hipStream_t st);
void launch_arc_src(const uint32_t *row_ptr, uint32_t V, uint32_t *arc_src, hipStream_t st);

// weight epochs: apply (arc, w) pairs to every weight array of the graph
void launch_weight_scatter(uint32_t n, const uint32_t *arc, const uint32_t *neww, uint32_t *w,
                           uint32_t *in_w, const uint32_t *in_pos, uint32_t *l_arc, uint32_t *x_w,
                           const uint32_t *arc_slot, uint32_t *li_arc, const uint32_t *arc_slot_in,
                           hipStream_t st);

// --------------------------------------------------------------- host side
// seg: caller's segments (nseg of them); sub (optional): a finer partition
// nested in the segments whose parts become the tiles (still cut to the cap).
void build_tiles(wr_graph *g, const uint32_t *seg, uint32_t nseg, uint32_t tile_cap,
                 bool bfs_grow, const uint32_t *sub = nullptr, uint32_t nsub = 0);
// Sort keys of the tiles for grouping sources into blocks: for a grid
// segmentation, the position of the tile's centroid cell along Hilbert's
// curve, per level, so that consecutive tiles form compact patches;
// otherwise the tile id.  Computed on first use and kept with the tiles.
const std::vector<uint64_t> &tile_order_keys(wr_graph *g);
// Rank of each tile in (key, tile) order.
const std::vector<uint32_t> &tile_order_rank(wr_graph *g);
void rebuild_tiles_if_needed(wr_graph *g);

}  // namespace wr
