// Schedule autotuner: times the supported (tile size, waves per workgroup,
// passes per graph replay) candidates on this graph with a deterministic set
// of sources and keeps the fastest.  Every candidate reaches the same exact
// fixpoint, so the choice changes speed only.  A JSON cache keyed by the
// graph's structure (CSR arrays and segmentation, not its weights) lets a
// later process reuse the choice without timing.
#include <chrono>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "wr_internal.hpp"

using namespace wr;

namespace {

struct Candidate {
    uint32_t tile, waves, passes;
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
    unsigned long long v_sig = 0, t = 0, w = 0, p = 0;
    if (!read_field(s, "signature", v_sig) || !read_field(s, "tile_vertices", t) ||
        !read_field(s, "waves_per_group", w) || !read_field(s, "passes_per_replay", p))
        return false;
    if (v_sig != sig) return false;
    c = Candidate{static_cast<uint32_t>(t), static_cast<uint32_t>(w), static_cast<uint32_t>(p)};
    return true;
}

void save_cache(const char *path, const wr_graph *g, uint64_t sig, const Candidate &c, double ms) {
    std::ofstream f(path, std::ios::trunc);
    if (!f) fail(WR_E_INVALID, std::string("cannot write autotune cache ") + path);
    f << "{\"signature\": \"" << sig << "\", \"V\": " << g->V << ", \"E\": " << g->E
      << ", \"tile_vertices\": " << c.tile << ", \"waves_per_group\": " << c.waves
      << ", \"passes_per_replay\": " << c.passes << ", \"ms\": " << ms << "}\n";
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

double time_candidate(wr_graph *g, const Candidate &c, const std::vector<uint32_t> &src,
                      std::vector<uint32_t> &out) {
    if (wr_graph_set_schedule(g, c.tile, c.waves, c.passes) != WR_OK) return -1;
    const uint32_t off[2] = {0, static_cast<uint32_t>(src.size())};
    double best = -1;
    for (int rep = 0; rep < 3; ++rep) {   // the first run builds tables and captures graphs
        const auto t0 = std::chrono::steady_clock::now();
        const wr_status st = wr_order_matrices(g, 1, off, src.data(), out.data(), nullptr, 0u, nullptr);
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
        const wr_status st = wr_graph_set_schedule(g, best.tile, best.waves, best.passes);
        if (st == WR_OK) return WR_OK;
    }
    const std::vector<uint32_t> src = tuning_sources(g, sources_hint ? sources_hint : 256u);
    if (src.empty()) return WR_OK;
    std::vector<uint32_t> out(src.size() * src.size());
    const Candidate prev{g->tile_vertices, g->waves_per_group, g->passes_per_replay};
    static const Candidate cands[] = {
        {256, 8, 8}, {512, 8, 8}, {512, 16, 8}, {256, 16, 8}, {512, 8, 4}, {512, 8, 16}, {256, 8, 16},
    };
    double best_ms = -1;
    for (const Candidate &c : cands) {
        const double ms = time_candidate(g, c, src, out);
        if (ms >= 0 && (best_ms < 0 || ms < best_ms)) {
            best_ms = ms;
            best = c;
        }
    }
    if (best_ms < 0) {
        (void)wr_graph_set_schedule(g, prev.tile, prev.waves, prev.passes);
        fail(WR_E_DEVICE, "no schedule candidate ran");
    }
    if (wr_graph_set_schedule(g, best.tile, best.waves, best.passes) != WR_OK)
        fail(WR_E_INTERNAL, "autotuner could not apply its choice");
    if (cache_path) save_cache(cache_path, g, sig, best, best_ms);
    WR_API_END
}
