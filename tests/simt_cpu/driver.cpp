// Runs one wr_sssp / wr_order_matrices request read from a file through the
// C ABI under the CPU executor -- TEST INFRASTRUCTURE ONLY.  Mode 2 sends
// the orders through the request server instead, one every `flags`
// milliseconds, so later orders arrive while earlier ones are relaxing.
// Mode 5 runs wr_wms_run (no graph).
//   wr_cpu_driver <request.bin> <result.bin>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "wroute.h"

static std::vector<uint32_t> g_in;
static size_t g_pos = 0;
static uint32_t rd() { return g_in.at(g_pos++); }
static std::vector<uint32_t> rdv(size_t n) {
    std::vector<uint32_t> v(g_in.begin() + g_pos, g_in.begin() + g_pos + n);
    g_pos += n;
    return v;
}

// wr_wms_run: params, runs, iters, A, M, orders, qty -> status, A, M,
// silhouette and area (two words per double), moves
static int run_wms(const char *outpath) {
    wr_wms_params p{};
    p.nx = rd();
    p.ny = rd();
    p.nz = rd();
    p.n_articles = rd();
    p.mmax = rd();
    p.purchase_orders = rd();
    p.articles_per_order = rd();
    p.clusters = rd();
    const uint32_t runs = rd(), iters = rd();
    const size_t V = static_cast<size_t>(p.nx) * p.ny * p.nz, S = static_cast<size_t>(p.purchase_orders) * p.articles_per_order;
    auto A = rdv(runs * V), M = rdv(runs * V), ord = rdv(runs * iters * S), qty = rdv(runs * iters * S);
    std::vector<double> sil(static_cast<size_t>(runs) * iters), area(sil.size());
    std::vector<uint32_t> mv(sil.size());
    wr_context *ctx = nullptr;
    wr_status st = wr_context_create(0, 0, &ctx);
    if (st == WR_OK)
        st = wr_wms_run(ctx, &p, runs, iters, A.data(), M.data(), ord.data(), qty.data(), sil.data(), area.data(),
                        mv.data(), 0, nullptr);
    if (st != WR_OK) std::fprintf(stderr, "status %s: %s\n", wr_status_str(st), wr_last_error());
    FILE *o = std::fopen(outpath, "wb");
    const uint32_t s32 = st;
    std::fwrite(&s32, 4, 1, o);
    std::fwrite(A.data(), 4, A.size(), o);
    std::fwrite(M.data(), 4, M.size(), o);
    std::fwrite(sil.data(), 8, sil.size(), o);
    std::fwrite(area.data(), 8, area.size(), o);
    std::fwrite(mv.data(), 4, mv.size(), o);
    std::fclose(o);
    wr_context_destroy(ctx);
    return 0;
}

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    uint32_t x;
    while (std::fread(&x, 4, 1, f) == 1) g_in.push_back(x);
    std::fclose(f);
    if (rd() != 0x57524F55u) return 2;
    const uint32_t mode = rd(), flags = rd(), want_pred = rd();
    if (mode == 5) return run_wms(argv[2]);
    const uint32_t V = rd(), E = rd();
    auto row_ptr = rdv(V + 1), col = rdv(E), w = rdv(E);
    wr_context *ctx = nullptr;
    wr_graph *g = nullptr;
    std::vector<uint32_t> out;
    std::vector<int32_t> pred;
    wr_status st = wr_context_create(0, 0, &ctx);
    if (st == WR_OK) st = wr_graph_create_csr(ctx, V, E, row_ptr.data(), col.data(), w.data(), 0, &g);
    const uint32_t seg_mode = rd();
    if (seg_mode == 1) {
        const uint32_t W = rd(), H = rd(), L = rd(), tw = rd(), th = rd();
        if (st == WR_OK) st = wr_graph_segment_grid(g, W, H, L, tw, th);
    } else if (seg_mode == 2) {
        const uint32_t ns = rd();
        auto m = rdv(V);
        if (st == WR_OK) st = wr_graph_set_segments(g, m.data(), ns);
    }
    const uint32_t tv = rd(), wv = rd(), kp = rd();
    if (st == WR_OK && (tv || wv || kp)) st = wr_graph_set_schedule(g, tv, wv, kp);
    const uint32_t nup = rd();
    auto ua = rdv(nup), uv = rdv(nup);
    if (st == WR_OK && nup) st = wr_graph_update_weights(g, nup, ua.data(), uv.data(), nullptr);
    if (mode == 0) {
        const uint32_t S = rd();
        auto src = rdv(S);
        out.assign(static_cast<size_t>(S) * V, 0);
        if (want_pred) pred.assign(static_cast<size_t>(S) * V, 0);
        if (st == WR_OK)
            st = wr_sssp(g, S, src.data(), out.data(), want_pred ? pred.data() : nullptr, flags, nullptr);
    } else if (mode == 2) {
        const uint32_t no = rd();
        auto off = rdv(no + 1);
        auto picks = rdv(off[no]);
        // weight updates: count, then per update its arcs, weights and the
        // number of orders submitted before it
        const uint32_t nupd = rd();
        std::vector<std::vector<uint32_t>> ua_(nupd), uw_(nupd);
        std::vector<uint32_t> after(nupd);
        for (uint32_t k = 0; k < nupd; ++k) {
            const uint32_t n = rd();
            ua_[k] = rdv(n);
            uw_[k] = rdv(n);
            after[k] = rd();
        }
        wr_server *srv = nullptr;
        wr_server_opts opts{};
        opts.max_source_slots = 128;
        opts.resident_epochs = nupd ? 2 : 1;
        if (st == WR_OK) st = wr_server_create(g, &opts, &srv);
        std::vector<uint64_t> tickets(no);
        for (uint32_t o = 0; o < no && st == WR_OK; ++o) {
            for (uint32_t k = 0; k < nupd && st == WR_OK; ++k)
                if (after[k] == o)
                    st = wr_server_update_weights(srv, static_cast<uint32_t>(ua_[k].size()), ua_[k].data(),
                                                  uw_[k].data());
            if (st == WR_OK) st = wr_server_submit(srv, off[o + 1] - off[o], picks.data() + off[o], &tickets[o]);
            // the first order is done before the others arrive (the server's
            // rows are built by then)
            if (st == WR_OK && o == 0 && nupd) st = wr_server_drain(srv);
            std::this_thread::sleep_for(std::chrono::milliseconds(flags));
        }
        if (st == WR_OK) st = wr_server_drain(srv);
        std::vector<uint32_t> epochs;
        for (uint32_t o = 0; o < no && st == WR_OK; ++o) {
            const uint32_t P = off[o + 1] - off[o];
            std::vector<uint32_t> m(static_cast<size_t>(P) * P);
            wr_req_info info{};
            st = wr_server_poll(srv, tickets[o], m.data(), &info);
            out.insert(out.end(), m.begin(), m.end());
            epochs.push_back(static_cast<uint32_t>(info.epoch));
        }
        out.insert(out.end(), epochs.begin(), epochs.end());
        wr_stats ss{};
        if (srv) wr_server_stats(srv, &ss);
        std::fprintf(stderr, "server: completed %llu steps %llu max_inflight %u\n",
                     static_cast<unsigned long long>(ss.completed), static_cast<unsigned long long>(ss.steps),
                     ss.max_inflight_requests);
        wr_server_destroy(srv);
    } else {
        const uint32_t no = rd();
        auto off = rdv(no + 1);
        auto picks = rdv(off[no]);
        // mode 4: cluster count and pick positions follow the picks
        const uint32_t m = mode == 4 ? rd() : 0;
        auto xyu = mode == 4 ? rdv(2 * off[no]) : std::vector<uint32_t>();
        size_t total = 0;
        for (uint32_t o = 0; o < no; ++o) total += static_cast<size_t>(off[o + 1] - off[o]) * (off[o + 1] - off[o]);
        out.assign(total, 0);
        if (want_pred) pred.assign(static_cast<size_t>(off[no]) * V, 0);
        if (st == WR_OK)
            st = wr_order_matrices(g, no, off.data(), picks.data(), out.data(),
                                   want_pred ? pred.data() : nullptr, flags, nullptr);
        if (mode == 4) {
            // clustered routes over the matrices just computed: lengths (two
            // words each), orderings, clusters used
            std::vector<uint64_t> len(no);
            std::vector<uint32_t> rt(off[no]), used(no);
            std::vector<int32_t> xy(xyu.begin(), xyu.end());
            if (st == WR_OK)
                st = wr_order_routes_clustered(ctx, no, off.data(), out.data(), xy.data(), m, len.data(), rt.data(),
                                               used.data(), 0, nullptr);
            for (uint64_t l : len) {
                out.push_back(static_cast<uint32_t>(l));
                out.push_back(static_cast<uint32_t>(l >> 32));
            }
            out.insert(out.end(), rt.begin(), rt.end());
            out.insert(out.end(), used.begin(), used.end());
        }
        if (mode == 3) {
            // routes over the matrices just computed: lengths (two words
            // each, low first) and orderings follow the matrices
            std::vector<uint64_t> len(no);
            std::vector<uint32_t> rt(off[no]);
            if (st == WR_OK) st = wr_order_routes(ctx, no, off.data(), out.data(), len.data(), rt.data(), 0, nullptr);
            for (uint64_t l : len) {
                out.push_back(static_cast<uint32_t>(l));
                out.push_back(static_cast<uint32_t>(l >> 32));
            }
            out.insert(out.end(), rt.begin(), rt.end());
        }
    }
    if (st != WR_OK) std::fprintf(stderr, "status %s: %s\n", wr_status_str(st), wr_last_error());
    FILE *o = std::fopen(argv[2], "wb");
    const uint32_t s32 = st;
    std::fwrite(&s32, 4, 1, o);
    std::fwrite(out.data(), 4, out.size(), o);
    if (!pred.empty()) std::fwrite(pred.data(), 4, pred.size(), o);
    std::fclose(o);
    wr_graph_destroy(g);
    wr_context_destroy(ctx);
    return 0;
}
