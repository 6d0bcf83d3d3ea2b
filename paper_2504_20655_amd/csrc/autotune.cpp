// Schedule autotuner: times schedule candidates on this graph with a
// deterministic set of sources and keeps the fastest.  With a grid
// segmentation the candidates are grid tile shapes (the segment rectangles
// the overlay tabulates), then the source blocks per workgroup unit, then
// the passes per graph replay, each stage around the best of the previous;
// otherwise (tile size, waves per workgroup, passes per replay).  Every
// candidate reaches the same exact fixpoint, so the choice changes speed
// only.  A JSON cache keyed by the graph's structure (CSR arrays and the
// segmentation the tuner was called with, not its weights) lets a later
// process reuse the choice without timing.
#include <chrono>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "wr_internal.hpp"

using namespace wr;

namespace {

constexpr uint32_t kTunePicks = 16;   // picks per synthetic order of a tuning solve

struct Candidate {
    uint32_t tile, waves, passes;
    uint32_t G = 0, tw = 0, th = 0;   // blocks per unit (0 = default); grid shape (0 = keep)
};

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Structure signature: CSR arrays and the caller's segmentation.
uint64_t signature(const wr_graph *g) {
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &g->V, sizeof g->V);
    h = fnv1a(h, &g->E, sizeof g->E);
    h = fnv1a(h, g->row_ptr.data(), g->row_ptr.size() * 4);
    h = fnv1a(h, g->col.data(), g->col.size() * 4);
    const uint32_t grid[6] = {g->tiles_user ? 1u : 0u, g->grid_W, g->grid_H, g->grid_L, g->grid_tw, g->grid_th};
    h = fnv1a(h, grid, sizeof grid);
    if (!g->user_seg.empty()) h = fnv1a(h, g->user_seg.data(), g->user_seg.size() * 4);
    return h;
}

// Minimal reader for the cache written below: one flat JSON object.
bool read_field(const std::string &s, const char *key, unsigned long long &v) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = s.find(k);
    if (p == std::string::npos) return false;
    p = s.find(':', p + k.size());
    if (p == std::string::npos) return false;
    ++p;
    while (p < s.size() && (s[p] == ' ' || s[p] == '"')) ++p;
    char *end = nullptr;
    v = std::strtoull(s.c_str() + p, &end, 10);
    return end != s.c_str() + p;
}

bool load_cache(const char *path, uint64_t sig, Candidate &c) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    unsigned long long v_sig = 0, t = 0, w = 0, p = 0, G = 0, tw = 0, th = 0;
    if (!read_field(s, "signature", v_sig) || !read_field(s, "tile_vertices", t) ||
        !read_field(s, "waves_per_group", w) || !read_field(s, "passes_per_replay", p))
        return false;
    if (v_sig != sig) return false;
    (void)read_field(s, "blocks_per_unit", G);
    (void)read_field(s, "grid_tile_w", tw);
    (void)read_field(s, "grid_tile_h", th);
    c = Candidate{static_cast<uint32_t>(t), static_cast<uint32_t>(w), static_cast<uint32_t>(p),
                  static_cast<uint32_t>(G), static_cast<uint32_t>(tw), static_cast<uint32_t>(th)};
    return true;
}

void save_cache(const char *path, const wr_graph *g, uint64_t sig, const Candidate &c, double ms) {
    std::ofstream f(path, std::ios::trunc);
    if (!f) fail(WR_E_INVALID, std::string("cannot write autotune cache ") + path);
    f << "{\"signature\": \"" << sig << "\", \"V\": " << g->V << ", \"E\": " << g->E
      << ", \"tile_vertices\": " << c.tile << ", \"waves_per_group\": " << c.waves
      << ", \"passes_per_replay\": " << c.passes << ", \"blocks_per_unit\": " << c.G
      << ", \"grid_tile_w\": " << c.tw << ", \"grid_tile_h\": " << c.th << ", \"ms\": " << ms << "}\n";
    if (!f) fail(WR_E_INVALID, std::string("cannot write autotune cache ") + path);
}

// Deterministic, well-spread sources: vertices with at least one arc at
// evenly spaced ids.
std::vector<uint32_t> tuning_sources(const wr_graph *g, uint32_t n) {
    std::vector<uint32_t> src;
    if (g->V == 0) return src;
    n = std::min(n, g->V);
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t v = static_cast<uint32_t>((static_cast<uint64_t>(i) * g->V) / n);
        for (uint32_t k = 0; k < g->V; ++k) {
            const uint32_t x = (v + k) % g->V;
            if (g->row_ptr[x + 1] > g->row_ptr[x]) {
                v = x;
                break;
            }
        }
        src.push_back(v);
    }
    return src;
}

// Puts candidate c in place: grid shape first (it rebuilds the tiles), then
// the schedule (which drops the cached work buffers).
wr_status apply(wr_graph *g, const Candidate &c) {
    if (c.tw && c.th && (c.tw != g->grid_tw || c.th != g->grid_th || !g->tiles)) {
        const wr_status st = wr_graph_segment_grid(g, g->grid_W, g->grid_H, g->grid_L, c.tw, c.th);
        if (st != WR_OK) return st;
    }
    const wr_status st = wr_graph_set_schedule(g, c.tile, c.waves, c.passes);
    if (st != WR_OK) return st;
    g->sources_per_unit = c.G;
    return WR_OK;
}

double time_candidate(wr_graph *g, const Candidate &c, const std::vector<uint32_t> &src,
                      std::vector<uint32_t> &out) {
    if (apply(g, c) != WR_OK) return -1;
    // the sources as orders of kTunePicks picks: the relaxation of every
    // source, read out into small matrices as a batch of orders is
    const uint32_t n = static_cast<uint32_t>(src.size());
    const uint32_t no = (n + kTunePicks - 1) / kTunePicks;
    std::vector<uint32_t> off(no + 1);
    for (uint32_t o = 0; o <= no; ++o) off[o] = std::min(n, o * kTunePicks);
    double best = -1;
    for (int rep = 0; rep < 4; ++rep) {   // the first run builds tables and captures graphs
        const auto t0 = std::chrono::steady_clock::now();
        const wr_status st = wr_order_matrices(g, no, off.data(), src.data(), out.data(), nullptr,
                                               g->grid_W ? WR_ALGO_OVERLAY : 0u, nullptr);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (st != WR_OK) return -1;
        if (rep > 0 && (best < 0 || ms < best)) best = ms;
    }
    return best;
}

}  // namespace

extern "C" wr_status wr_autotune(wr_graph *g, uint32_t sources_hint, const char *cache_path) {
    WR_API_BEGIN
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    const uint64_t sig = signature(g);
    Candidate best{};
    if (cache_path && load_cache(cache_path, sig, best)) {
        if (apply(g, best) == WR_OK) return WR_OK;
    }
    const std::vector<uint32_t> src = tuning_sources(g, sources_hint ? sources_hint : 256u);
    if (src.empty()) return WR_OK;
    std::vector<uint32_t> out(src.size() * kTunePicks);
    const Candidate prev{g->tile_vertices, g->waves_per_group, g->passes_per_replay, g->sources_per_unit,
                         g->grid_tw, g->grid_th};
    double best_ms = -1;
    auto consider = [&](const Candidate &c) {
        const double ms = time_candidate(g, c, src, out);
        if (ms >= 0 && (best_ms < 0 || ms < best_ms)) {
            best_ms = ms;
            best = c;
        }
    };
    if (g->grid_W) {
        // grid tile shapes around the caller's, each cut into tiles of at
        // most 512 vertices; shapes the overlay tables cannot hold fail to
        // run and drop out
        static const uint32_t shapes[][2] = {{24, 20}, {21, 24}, {12, 40}, {18, 40}, {15, 48}, {21, 32},
                                             {12, 60}, {24, 24}, {16, 32}, {32, 16}, {18, 24}};
        consider(Candidate{512, 8, 8, 4, g->grid_tw, g->grid_th});
        for (const auto &sh : shapes)
            if (sh[0] != prev.tw || sh[1] != prev.th) consider(Candidate{512, 8, 8, 4, sh[0], sh[1]});
        const Candidate shape = best;
        for (uint32_t G : {2u, 3u, 6u, 8u, 12u, 16u, 24u})
            consider(Candidate{shape.tile, shape.waves, shape.passes, G, shape.tw, shape.th});
        const Candidate unit = best;
        for (uint32_t K : {4u, 16u}) consider(Candidate{unit.tile, unit.waves, K, unit.G, unit.tw, unit.th});
    } else {
        static const Candidate cands[] = {
            {256, 8, 8}, {512, 8, 8}, {512, 16, 8}, {256, 16, 8}, {512, 8, 4}, {512, 8, 16}, {256, 8, 16},
        };
        for (const Candidate &c : cands) consider(c);
    }
    if (best_ms < 0) {
        (void)apply(g, prev);
        fail(WR_E_DEVICE, "no schedule candidate ran");
    }
    if (apply(g, best) != WR_OK) fail(WR_E_INTERNAL, "autotuner could not apply its choice");
    if (cache_path) save_cache(cache_path, g, sig, best, best_ms);
    WR_API_END
}

extern "C" wr_status wr_graph_get_schedule(const wr_graph *g, wr_schedule *out) {
    WR_API_BEGIN
    if (!g || !out) fail(WR_E_INVALID, "NULL argument");
    out->tile_vertices = g->tile_vertices;
    out->waves_per_group = g->waves_per_group;
    out->passes_per_replay = g->passes_per_replay;
    out->blocks_per_unit = g->sources_per_unit ? g->sources_per_unit : (g->lanes == 64 ? 4u : 4u * g->waves_per_group);
    out->grid_tile_w = g->grid_W ? g->grid_tw : 0u;
    out->grid_tile_h = g->grid_W ? g->grid_th : 0u;
    WR_API_END
}

extern "C" wr_status wr_graph_set_blocks_per_unit(wr_graph *g, uint32_t blocks) {
    WR_API_BEGIN
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    if (blocks > 64) fail(WR_E_INVALID, "at most 64 blocks per unit");
    g->sources_per_unit = blocks;
    destroy_workspace(g->ws);
    g->ws = nullptr;
    WR_API_END
}
