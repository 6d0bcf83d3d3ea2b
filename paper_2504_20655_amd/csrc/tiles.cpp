// Segment builder: turns a vertex -> segment map (or a grid tile spec, or an
// automatic breadth-first partition) into LDS tiles with boundary tables.
//
// A segment is a vertex set chosen by the caller; its boundary vertices are
// those with an arc to or from another segment.  The paper divides routing
// work into sub-problems processed independently within the GPU's memory
// (Discussion) and joins route pieces through boundary nodes (Route
// Optimization section, Theorem).  Here a segment is further cut into tiles
// small enough for one wave's LDS distance array; tiles are what the kernels
// relax.  Boundary-in vertices ("ports") receive values pushed from other
// tiles; boundary-out vertices push their cross-tile arcs.
#include <algorithm>
#include <memory>
#include <numeric>

#include "wr_internal.hpp"

namespace wr {

namespace {

// Sorted unique tile list helper: split the id-ordered vertex list of one
// segment into tiles of at most `cap` vertices whose summed out-degree stays
// within 4*cap (the LDS arc budget of a tile).
void cut_segment(const std::vector<uint32_t> &verts, const std::vector<uint32_t> &row_ptr,
                 uint32_t cap, std::vector<uint32_t> &tile_of, uint32_t &T) {
    uint32_t n = 0;
    uint64_t arcs = 0;
    bool open = false;
    for (uint32_t v : verts) {
        const uint32_t deg = row_ptr[v + 1] - row_ptr[v];
        if (!open || n + 1 > cap || arcs + deg > 4ull * cap) {
            ++T;
            n = 0;
            arcs = 0;
            open = true;
        }
        tile_of[v] = T - 1;
        ++n;
        arcs += deg;
    }
}

}  // namespace

void build_tiles(wr_graph *g, const uint32_t *seg, uint32_t nseg, uint32_t cap, bool bfs_grow,
                 const uint32_t *sub, uint32_t nsub) {
    const uint32_t V = g->V;
    const auto &row_ptr = g->row_ptr;
    const auto &col = g->col;
    const auto &w = g->w;

    // incident vertices
    std::vector<uint8_t> inc(V, 0);
    for (uint32_t u = 0; u < V; ++u)
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            inc[u] = 1;
            inc[col[e]] = 1;
        }
    for (uint32_t u = 0; u < V; ++u)
        if (row_ptr[u + 1] - row_ptr[u] > 4ull * cap)
            fail(WR_E_UNSUPPORTED, "a vertex has more out-arcs than one LDS tile holds");

    auto ts = std::make_unique<TileSet>();
    ts->tile_cap = cap;
    ts->tile_of.assign(V, NONE);
    uint32_t T = 0;
    if (bfs_grow) {
        // undirected adjacency through out- and in-arcs
        std::vector<uint32_t> in_ptr(V + 1, 0), in_src(g->E);
        for (uint32_t e = 0; e < g->E; ++e) in_ptr[col[e] + 1]++;
        for (uint32_t v = 0; v < V; ++v) in_ptr[v + 1] += in_ptr[v];
        {
            std::vector<uint32_t> fill(in_ptr.begin(), in_ptr.end() - 1);
            for (uint32_t u = 0; u < V; ++u)
                for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) in_src[fill[col[e]]++] = u;
        }
        std::vector<uint32_t> queue;
        queue.reserve(cap);
        for (uint32_t s = 0; s < V; ++s) {
            if (!inc[s] || ts->tile_of[s] != NONE) continue;
            const uint32_t t = T++;
            uint32_t n = 0;
            uint64_t arcs = 0;
            queue.clear();
            queue.push_back(s);
            ts->tile_of[s] = t;
            n = 1;
            arcs = row_ptr[s + 1] - row_ptr[s];
            for (size_t h = 0; h < queue.size(); ++h) {
                const uint32_t u = queue[h];
                auto try_add = [&](uint32_t x) {
                    if (n >= cap || ts->tile_of[x] != NONE || !inc[x]) return;
                    const uint32_t deg = row_ptr[x + 1] - row_ptr[x];
                    if (arcs + deg > 4ull * cap) return;
                    ts->tile_of[x] = t;
                    ++n;
                    arcs += deg;
                    queue.push_back(x);
                };
                for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) try_add(col[e]);
                for (uint32_t e = in_ptr[u]; e < in_ptr[u + 1]; ++e) try_add(in_src[e]);
            }
        }
        ts->num_segments = T;
    } else {
        // bucket incident vertices by part (the finer partition if given,
        // else the segment), id order inside a part, and cut parts to the cap
        const uint32_t *part = sub ? sub : seg;
        const uint32_t nparts = sub ? nsub : nseg;
        std::vector<uint32_t> cnt(nparts + 1, 0);
        for (uint32_t v = 0; v < V; ++v)
            if (inc[v]) cnt[part[v] + 1]++;
        for (uint32_t s = 0; s < nparts; ++s) cnt[s + 1] += cnt[s];
        std::vector<uint32_t> order(cnt[nparts]);
        {
            std::vector<uint32_t> fill(cnt.begin(), cnt.end() - 1);
            for (uint32_t v = 0; v < V; ++v)
                if (inc[v]) order[fill[part[v]]++] = v;
        }
        std::vector<uint32_t> verts;
        for (uint32_t s = 0; s < nparts; ++s) {
            verts.assign(order.begin() + cnt[s], order.begin() + cnt[s + 1]);
            cut_segment(verts, row_ptr, cap, ts->tile_of, T);
        }
        ts->num_segments = nseg;
    }
    ts->T = T;

    // positions: tile by tile, ascending vertex id inside a tile
    std::vector<uint32_t> tsize(T + 1, 0);
    for (uint32_t v = 0; v < V; ++v)
        if (ts->tile_of[v] != NONE) tsize[ts->tile_of[v] + 1]++;
    for (uint32_t t = 0; t < T; ++t) tsize[t + 1] += tsize[t];
    ts->tile_base = tsize;
    const uint32_t Vt = tsize[T];
    ts->Vt = Vt;
    ts->pos_of.assign(V, NONE);
    ts->vert_of.resize(Vt);
    {
        std::vector<uint32_t> fill(tsize.begin(), tsize.end() - 1);
        for (uint32_t v = 0; v < V; ++v) {
            const uint32_t t = ts->tile_of[v];
            if (t == NONE) continue;
            const uint32_t p = fill[t]++;
            ts->pos_of[v] = p;
            ts->vert_of[p] = v;
        }
    }

    // ports (boundary-in) and boundary-out vertices
    std::vector<uint8_t> is_port(Vt, 0), is_bout(Vt, 0);
    uint64_t cross = 0;
    for (uint32_t u = 0; u < V; ++u) {
        const uint32_t tu = ts->tile_of[u];
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const uint32_t x = col[e];
            if (ts->tile_of[x] != tu) {
                is_port[ts->pos_of[x]] = 1;
                is_bout[ts->pos_of[u]] = 1;
                ++cross;
            }
        }
    }
    ts->cross_arcs = cross;
    std::vector<uint32_t> port_id(Vt, NONE);
    ts->port_base.assign(T + 1, 0);
    ts->bo_base.assign(T + 1, 0);
    for (uint32_t t = 0; t < T; ++t) {
        ts->port_base[t + 1] = ts->port_base[t];
        ts->bo_base[t + 1] = ts->bo_base[t];
        for (uint32_t p = tsize[t]; p < tsize[t + 1]; ++p) {
            if (is_port[p]) {
                port_id[p] = ts->port_base[t + 1]++;
                ts->port_local.push_back(p - tsize[t]);
            }
            if (is_bout[p]) {
                ts->bo_base[t + 1]++;
                ts->bo_local.push_back(p - tsize[t]);
            }
        }
    }
    ts->NP = ts->port_base[T];
    ts->NB = ts->bo_base[T];
    for (uint32_t t = 0; t < T; ++t) {
        ts->max_ports = std::max(ts->max_ports, ts->port_base[t + 1] - ts->port_base[t]);
        ts->max_exits = std::max(ts->max_exits, ts->bo_base[t + 1] - ts->bo_base[t]);
    }

    // per-position arc lists
    ts->l_off.assign(Vt + 1, 0);
    ts->x_off.assign(Vt + 1, 0);
    ts->arc_slot.assign(g->E, NONE);
    for (uint32_t p = 0; p < Vt; ++p) {
        const uint32_t u = ts->vert_of[p];
        const uint32_t tu = ts->tile_of[u];
        uint32_t nl = 0, nx = 0;
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) (ts->tile_of[col[e]] == tu ? nl : nx)++;
        ts->l_off[p + 1] = ts->l_off[p] + nl;
        ts->x_off[p + 1] = ts->x_off[p] + nx;
    }
    ts->l_arc.resize(ts->l_off[Vt]);
    ts->x_port.resize(ts->x_off[Vt]);
    ts->x_w.resize(ts->x_off[Vt]);
    ts->x_tile.resize(ts->x_off[Vt]);
    for (uint32_t p = 0; p < Vt; ++p) {
        const uint32_t u = ts->vert_of[p];
        const uint32_t tu = ts->tile_of[u];
        uint32_t li = ts->l_off[p], xi = ts->x_off[p];
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const uint32_t x = col[e];
            const uint32_t tx = ts->tile_of[x];
            if (tx == tu) {
                const uint32_t loc = ts->pos_of[x] - tsize[tu];
                ts->l_arc[li] = (loc << 16) | (w[e] & 0xFFFFu);
                ts->arc_slot[e] = li++;
            } else {
                ts->x_port[xi] = port_id[ts->pos_of[x]];
                ts->x_w[xi] = w[e];
                ts->x_tile[xi] = tx;
                ts->arc_slot[e] = 0x80000000u | xi++;
            }
        }
    }
    for (uint32_t t = 0; t < T; ++t) {
        if (ts->l_off[tsize[t + 1]] - ts->l_off[tsize[t]] > 4ull * cap)
            fail(WR_E_INTERNAL, "tile arc budget exceeded");
        ts->max_cross = std::max(ts->max_cross, ts->x_off[tsize[t + 1]] - ts->x_off[tsize[t]]);
    }
    {
        std::vector<uint32_t> in_cnt(T, 0u);
        for (uint32_t tx : ts->x_tile) in_cnt[tx]++;
        for (uint32_t t = 0; t < T; ++t) ts->max_cross_in = std::max(ts->max_cross_in, in_cnt[t]);
    }

    // in-tile in-arcs (pull form): the same arcs grouped by target position
    ts->li_off.assign(Vt + 1, 0);
    ts->arc_slot_in.assign(g->E, NONE);
    for (uint32_t p = 0; p < Vt; ++p) {
        const uint32_t u = ts->vert_of[p];
        const uint32_t tu = ts->tile_of[u];
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (ts->tile_of[col[e]] == tu) ts->li_off[ts->pos_of[col[e]] + 1]++;
    }
    for (uint32_t p = 0; p < Vt; ++p) ts->li_off[p + 1] += ts->li_off[p];
    ts->li_arc.resize(ts->li_off[Vt]);
    {
        std::vector<uint32_t> fill(ts->li_off.begin(), ts->li_off.end() - 1);
        for (uint32_t p = 0; p < Vt; ++p) {
            const uint32_t u = ts->vert_of[p];
            const uint32_t tu = ts->tile_of[u];
            const uint32_t uloc = p - tsize[tu];
            for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                if (ts->tile_of[col[e]] != tu) continue;
                const uint32_t q = fill[ts->pos_of[col[e]]]++;
                ts->li_arc[q] = (uloc << 16) | (w[e] & 0xFFFFu);
                ts->arc_slot_in[e] = q;
            }
        }
    }

    // upload
    wr_context *ctx = g->ctx;
    hipStream_t st = ctx->stream;
    upload(ts->d_tile_of, ctx, ts->tile_of, st);
    upload(ts->d_pos_of, ctx, ts->pos_of, st);
    upload(ts->d_tile_base, ctx, ts->tile_base, st);
    upload(ts->d_l_off, ctx, ts->l_off, st);
    upload(ts->d_l_arc, ctx, ts->l_arc, st);
    upload(ts->d_x_off, ctx, ts->x_off, st);
    upload(ts->d_x_port, ctx, ts->x_port, st);
    upload(ts->d_x_w, ctx, ts->x_w, st);
    upload(ts->d_x_tile, ctx, ts->x_tile, st);
    upload(ts->d_port_base, ctx, ts->port_base, st);
    upload(ts->d_port_local, ctx, ts->port_local, st);
    upload(ts->d_bo_base, ctx, ts->bo_base, st);
    upload(ts->d_bo_local, ctx, ts->bo_local, st);
    upload(ts->d_arc_slot, ctx, ts->arc_slot, st);
    upload(ts->d_li_off, ctx, ts->li_off, st);
    upload(ts->d_li_arc, ctx, ts->li_arc, st);
    upload(ts->d_arc_slot_in, ctx, ts->arc_slot_in, st);
    WR_HIP(hipStreamSynchronize(st));
    destroy_workspace(g->ws);
    g->ws = nullptr;
    delete g->tiles;
    g->tiles = ts.release();
    g->tiles_gen += 1;
}

namespace {

// Interior cut positions along one axis of extent n: segments of `seg`
// cells from 0, each cut into pieces of about `sub` cells.  A piece boundary
// moves by up to a quarter piece (at most 2 cells) to the boundary the
// fewest arcs cross (cross[c] = arcs between cell c-1 and c, ties to the
// nominal position), so cuts avoid splitting corridors the arcs run along.
// Returns, per cell, its piece index inside its segment.
std::vector<uint32_t> grid_cuts(uint32_t n, uint32_t seg, uint32_t sub, const std::vector<uint64_t> &cross) {
    std::vector<uint32_t> piece(n, 0);
    const uint32_t r = std::min(2u, sub / 4);
    for (uint32_t s0 = 0; s0 < n; s0 += seg) {
        const uint32_t s1 = std::min(n, s0 + seg);
        uint32_t prev = s0, k = 0;
        for (uint32_t c = s0 + sub; c < s1; c += sub) {
            uint32_t best = c;
            for (uint32_t d = 1; d <= r; ++d) {
                for (uint32_t cand : {c - d, c + d}) {
                    if (cand <= prev || cand >= s1) continue;
                    if (cross[cand] < cross[best]) best = cand;
                }
            }
            for (uint32_t x = prev; x < best; ++x) piece[x] = k;
            prev = best;
            ++k;
        }
        for (uint32_t x = prev; x < s1; ++x) piece[x] = k;
    }
    return piece;
}

// Grid segments (tile_w x tile_h cells per level) and, nested in them,
// sub-rectangles holding at most `cap` vertices incident to an arc (blocked
// cells are isolated ids and take no tile space): halve the longer side of
// the sub-rectangle until every one of them fits, with the sub-rectangles'
// boundaries snapped to the rows and columns the fewest arcs cross.
void grid_maps(const wr_graph *g, uint32_t W, uint32_t H, uint32_t L, uint32_t tw, uint32_t th, uint32_t cap,
               std::vector<uint32_t> &seg, uint32_t &nseg, std::vector<uint32_t> &sub, uint32_t &nsub) {
    const uint32_t tx = (W + tw - 1) / tw, ty = (H + th - 1) / th;
    const size_t plane = static_cast<size_t>(W) * H;
    std::vector<uint8_t> inc(plane * L, 0);
    std::vector<uint64_t> crossx(W + 1, 0), crossy(H + 1, 0);
    for (uint32_t u = 0; u < g->V; ++u)
        for (uint32_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; ++e) {
            const uint32_t v = g->col[e];
            inc[u] = 1;
            inc[v] = 1;
            if (u / plane != v / plane) continue;
            const uint32_t ux = (u % plane) % W, uy = static_cast<uint32_t>((u % plane) / W);
            const uint32_t vx = (v % plane) % W, vy = static_cast<uint32_t>((v % plane) / W);
            if (uy == vy && (ux + 1 == vx || vx + 1 == ux)) crossx[std::max(ux, vx)]++;
            if (ux == vx && (uy + 1 == vy || vy + 1 == uy)) crossy[std::max(uy, vy)]++;
        }
    std::vector<uint32_t> px, py;
    auto fits = [&](uint32_t sw, uint32_t sh) {
        px = grid_cuts(W, tw, sw, crossx);
        py = grid_cuts(H, th, sh, crossy);
        const uint32_t sx = (tw + sw - 1) / sw + 1, sy = (th + sh - 1) / sh + 1;
        const uint64_t n = static_cast<uint64_t>(tx) * ty * L * sx * sy;
        std::vector<uint32_t> cnt(n, 0u);
        for (uint32_t l = 0; l < L; ++l)
            for (uint32_t y = 0; y < H; ++y)
                for (uint32_t x = 0; x < W; ++x) {
                    const size_t v = l * plane + static_cast<size_t>(y) * W + x;
                    if (!inc[v]) continue;
                    const uint64_t s = (static_cast<uint64_t>(l) * ty + y / th) * tx + x / tw;
                    const uint64_t q = (s * sy + py[y]) * sx + px[x];
                    if (++cnt[q] > cap) return false;
                }
        return true;
    };
    uint32_t sw = tw, sh = th;
    while ((sw > 1 || sh > 1) && !fits(sw, sh)) {
        if (sw >= sh) sw = (sw + 1) / 2;
        else sh = (sh + 1) / 2;
    }
    // a snapped piece can be up to 2 cells wider than sw: one spare index
    const uint32_t sx = (tw + sw - 1) / sw + 1, sy = (th + sh - 1) / sh + 1;
    nseg = tx * ty * L;
    nsub = nseg * sx * sy;
    seg.resize(plane * L);
    sub.resize(seg.size());
    for (uint32_t l = 0; l < L; ++l)
        for (uint32_t y = 0; y < H; ++y)
            for (uint32_t x = 0; x < W; ++x) {
                const size_t v = l * plane + static_cast<size_t>(y) * W + x;
                const uint32_t s = (l * ty + y / th) * tx + x / tw;
                seg[v] = s;
                sub[v] = (s * sy + py[y]) * sx + px[x];
            }
}

}  // namespace

namespace {
// Position of cell (x, y) along Hilbert's curve over the n x n grid (n a
// power of two above both coordinates): at every level the quadrant the
// point falls in contributes its rank along the curve (lower left, upper
// left, upper right, lower right), and the point is then mapped into that
// quadrant's frame (the lower quadrants are traversed transposed, the lower
// right one also mirrored), so consecutive positions are always adjacent
// cells and a run of positions stays compact.
uint64_t hilbert2(uint32_t n, uint32_t x, uint32_t y) {
    uint64_t d = 0;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += static_cast<uint64_t>(s) * s * ((3u * rx) ^ ry);
        x &= s - 1;
        y &= s - 1;
        if (ry == 0) {
            if (rx == 1) {
                x = s - 1 - x;
                y = s - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}
}  // namespace

const std::vector<uint64_t> &tile_order_keys(wr_graph *g) {
    TileSet &ts = *g->tiles;
    if (ts.order_key.size() == ts.T) return ts.order_key;
    ts.order_key.assign(ts.T, 0);
    const uint64_t plane = static_cast<uint64_t>(g->grid_W) * g->grid_H;
    const bool grid = g->tiles_user && g->grid_W && g->grid_H &&
                      plane * std::max(g->grid_L, 1u) == static_cast<uint64_t>(g->V);
    uint32_t side = 1;   // a power of two above both grid dimensions
    while (side < std::max(g->grid_W, g->grid_H)) side <<= 1;
    for (uint32_t t = 0; t < ts.T; ++t) {
        if (!grid) {
            ts.order_key[t] = t;
            continue;
        }
        uint64_t sx = 0, sy = 0, n = 0, lv = 0;
        for (uint32_t p = ts.tile_base[t]; p < ts.tile_base[t + 1]; ++p) {
            const uint64_t v = ts.vert_of[p];
            const uint64_t r = v % plane;
            sx += r % g->grid_W;
            sy += r / g->grid_W;
            lv = v / plane;
            ++n;
        }
        const uint32_t cx = n ? static_cast<uint32_t>(sx / n) : 0, cy = n ? static_cast<uint32_t>(sy / n) : 0;
        ts.order_key[t] = (lv << 42) | hilbert2(side, cx, cy);
    }
    return ts.order_key;
}

const std::vector<uint32_t> &tile_order_rank(wr_graph *g) {
    TileSet &ts = *g->tiles;
    if (ts.order_rank.size() == ts.T) return ts.order_rank;
    const std::vector<uint64_t> &key = tile_order_keys(g);
    std::vector<uint32_t> by(ts.T);
    for (uint32_t t = 0; t < ts.T; ++t) by[t] = t;
    std::sort(by.begin(), by.end(), [&](uint32_t a, uint32_t b) { return key[a] != key[b] ? key[a] < key[b] : a < b; });
    ts.order_rank.assign(ts.T, 0u);
    for (uint32_t r = 0; r < ts.T; ++r) ts.order_rank[by[r]] = r;
    return ts.order_rank;
}

void rebuild_tiles_if_needed(wr_graph *g) {
    if (g->tiles && g->tiles->tile_cap == g->tile_vertices) return;
    if (g->grid_W) {
        std::vector<uint32_t> seg, sub;
        uint32_t nseg, nsub;
        grid_maps(g, g->grid_W, g->grid_H, g->grid_L, g->grid_tw, g->grid_th, g->tile_vertices, seg, nseg, sub,
                  nsub);
        build_tiles(g, seg.data(), nseg, g->tile_vertices, false, sub.data(), nsub);
    } else if (g->tiles_user) {
        build_tiles(g, g->user_seg.data(), g->user_num_segments, g->tile_vertices, false);
    } else {
        build_tiles(g, nullptr, 0, g->tile_vertices, true);
    }
}

}  // namespace wr

using namespace wr;

extern "C" {

wr_status wr_graph_set_segments(wr_graph *g, const uint32_t *segment_of_vertex,
                                uint32_t num_segments) {
    WR_API_BEGIN
    if (!g || !segment_of_vertex) fail(WR_E_INVALID, "NULL argument");
    if (num_segments == 0) fail(WR_E_INVALID, "num_segments must be positive");
    for (uint32_t v = 0; v < g->V; ++v)
        if (segment_of_vertex[v] >= num_segments) fail(WR_E_INVALID, "segment id out of range");
    WR_HIP(hipSetDevice(g->ctx->device));
    std::vector<uint32_t> seg(segment_of_vertex, segment_of_vertex + g->V);
    build_tiles(g, seg.data(), num_segments, g->tile_vertices, false);
    g->user_seg.swap(seg);
    g->user_num_segments = num_segments;
    g->tiles_user = true;
    g->grid_W = 0;
    WR_API_END
}

wr_status wr_graph_segment_grid(wr_graph *g, uint32_t W, uint32_t H, uint32_t levels,
                                uint32_t tile_w, uint32_t tile_h) {
    WR_API_BEGIN
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    if (!W || !H || !levels || !tile_w || !tile_h) fail(WR_E_INVALID, "sizes must be positive");
    if (static_cast<uint64_t>(W) * H * levels != g->V) fail(WR_E_INVALID, "W*H*levels != V");
    const uint64_t nseg64 = static_cast<uint64_t>((W + tile_w - 1) / tile_w) * ((H + tile_h - 1) / tile_h) * levels;
    if (nseg64 >= 0xFFFFFFFFull / 4) fail(WR_E_INVALID, "too many segments");
    WR_HIP(hipSetDevice(g->ctx->device));
    std::vector<uint32_t> seg, sub;
    uint32_t nseg, nsub;
    grid_maps(g, W, H, levels, tile_w, tile_h, g->tile_vertices, seg, nseg, sub, nsub);
    build_tiles(g, seg.data(), nseg, g->tile_vertices, false, sub.data(), nsub);
    g->user_seg.swap(seg);
    g->user_num_segments = nseg;
    g->tiles_user = true;
    g->grid_W = W;
    g->grid_H = H;
    g->grid_L = levels;
    g->grid_tw = tile_w;
    g->grid_th = tile_h;
    WR_API_END
}

wr_status wr_graph_segment_info(const wr_graph *g, uint32_t *num_segments, uint32_t *num_tiles,
                                uint32_t *num_boundary) {
    WR_API_BEGIN
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    const TileSet *ts = g->tiles;
    if (num_segments) *num_segments = ts ? ts->num_segments : 0;
    if (num_tiles) *num_tiles = ts ? ts->T : 0;
    if (num_boundary) *num_boundary = ts ? ts->NP : 0;
    WR_API_END
}

}  // extern "C"
