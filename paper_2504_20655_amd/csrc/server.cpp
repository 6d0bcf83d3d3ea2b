// Continuous-batching server.  Orders arrive at any time; a scheduler thread
// owns the GPU.  In the streaming mode (graphs whose tiling runs the overlay
// schedule) the device holds a fixed set of block rows of 64 source lanes.
// Each scheduler step admits queued orders into free rows (their distinct
// picks seeded while the other rows keep relaxing), replays one group of
// relaxation passes over every row, retires the orders whose rows have all
// converged (their P x P matrices gathered and copied to the host) and frees
// rows no order uses any more.  Other graphs fall back to step batching: the
// admitted orders are solved together in one multi-source call.
//
// Weight updates queue; admission pauses until the rows in flight have
// converged, then the update is applied, so every order is solved entirely
// on the epoch current at its admission.  An order's matrix is the same alone
// or in any mix, because every schedule reaches the exact fixpoint.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wr_internal.hpp"

using namespace wr;

namespace {

double clock_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    std::vector<uint32_t> picks;
    std::vector<uint32_t> dist;   // P x P once done
    wr_req_info info{};
    bool done = false;
};

struct WeightBatch {
    std::vector<uint32_t> arc, w;
};

}  // namespace

struct wr_server {
    wr_graph *g = nullptr;
    wr_server_opts opts{};
    uint64_t budget = 0;              // device bytes an admitted batch may take
    std::mutex mu;
    std::condition_variable cv_work;  // scheduler: new requests, updates or stop
    std::condition_variable cv_done;  // drain / poll waiters
    std::deque<Request *> queue;      // submitted, not admitted
    std::unordered_map<uint64_t, Request *> reqs;   // ticket -> request (until polled)
    std::deque<WeightBatch> updates;
    uint64_t next_ticket = 1;
    uint64_t outstanding = 0;         // submitted and not yet done
    bool stop = false;
    // statistics
    uint64_t submitted = 0, completed = 0, failed = 0, steps = 0;
    uint32_t max_inflight = 0;
    double first_arrive = -1, last_done = 0;
    std::vector<double> lat_ms;
    double t0 = 0;
    std::thread worker;
    // streaming mode
    StreamSolver *stream = nullptr;
    // phase timers (seconds), printed at destroy when WR_TRACE is set
    double t_update = 0, t_admit = 0, t_step = 0, t_gather = 0, t_wait = 0;
    uint64_t rows_admitted = 0;
};

namespace {

// Device bytes one admitted batch needs besides the graph: the output
// matrices plus the per-source relaxation state (rounded up to blocks of 64).
uint64_t batch_bytes(const wr_graph *g, uint64_t sources, uint64_t out_entries) {
    const TileSet *ts = g->tiles;
    const uint64_t blocks = (sources + 63) / 64;
    uint64_t per_block;
    if (ts)
        per_block = SegBuffers::bytes_per_row(*ts, 4, 64, false);
    else
        per_block = 64ull * 4ull * g->V * 2ull;
    return out_entries * 4ull + blocks * per_block + (8ull << 20);
}

void finish(wr_server *s, Request *r, wr_status st, double t_done) {
    r->info.status = st;
    r->info.t_done = t_done - s->t0;
    r->done = true;
    --s->outstanding;
    if (st == WR_OK) {
        ++s->completed;
        s->lat_ms.push_back((r->info.t_done - r->info.t_arrive) * 1e3);
        s->last_done = std::max(s->last_done, r->info.t_done);
    } else {
        ++s->failed;
    }
}

// Applies queued weight updates (caller: nothing in flight).
void apply_updates(wr_server *s, std::vector<WeightBatch> &ups) {
    for (WeightBatch &u : ups) {
        uint64_t ep = 0;
        const wr_status st = wr_graph_update_weights(s->g, static_cast<uint32_t>(u.arc.size()), u.arc.data(),
                                                     u.w.data(), &ep);
        if (st != WR_OK) set_last_error(std::string("server weight update rejected: ") + wr_status_str(st));
    }
    ups.clear();
}

// Step batching: every admitted order in one multi-source call.
void run_step_mode(wr_server *s) {
    const uint32_t slots = s->opts.max_source_slots;
    std::vector<Request *> batch;
    std::vector<uint32_t> off, picks, out;
    for (;;) {
        std::vector<WeightBatch> ups;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->updates.empty(); });
            if (s->stop && s->queue.empty() && s->updates.empty()) return;
            // weight updates apply between steps: nothing is in flight here
            while (!s->updates.empty()) {
                ups.push_back(std::move(s->updates.front()));
                s->updates.pop_front();
            }
        }
        apply_updates(s, ups);
        // admission: queued orders in arrival order while slots and memory allow
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(s->mu);
            uint64_t src = 0, outn = 0;
            const double now = clock_s() - s->t0;
            while (!s->queue.empty()) {
                Request *r = s->queue.front();
                const uint64_t P = r->picks.size();
                const uint64_t need = batch_bytes(s->g, src + P, outn + P * P);
                if (!batch.empty() && (src + P > slots || need > s->budget)) break;
                s->queue.pop_front();
                if (batch_bytes(s->g, P, P * P) > s->budget) {
                    // can never be admitted: fail it, keep serving the rest
                    r->info.t_admit = now;
                    finish(s, r, WR_E_NOMEM, clock_s());
                    s->cv_done.notify_all();
                    continue;
                }
                r->info.t_admit = now;
                r->info.epoch = s->g->epoch;
                batch.push_back(r);
                src += P;
                outn += P * P;
            }
            s->max_inflight = std::max<uint32_t>(s->max_inflight, static_cast<uint32_t>(batch.size()));
        }
        if (batch.empty()) continue;
        off.assign(1, 0u);
        picks.clear();
        for (Request *r : batch) {
            picks.insert(picks.end(), r->picks.begin(), r->picks.end());
            off.push_back(static_cast<uint32_t>(picks.size()));
        }
        uint64_t total = 0;
        for (Request *r : batch) total += static_cast<uint64_t>(r->picks.size()) * r->picks.size();
        out.resize(total);
        const wr_status st = wr_order_matrices(s->g, static_cast<uint32_t>(batch.size()), off.data(),
                                               picks.data(), out.data(), nullptr, 0u, nullptr);
        const double t_done = clock_s();
        std::unique_lock<std::mutex> lk(s->mu);
        ++s->steps;
        uint64_t at = 0;
        for (Request *r : batch) {
            const uint64_t n = static_cast<uint64_t>(r->picks.size()) * r->picks.size();
            if (st == WR_OK) r->dist.assign(out.begin() + at, out.begin() + at + n);
            at += n;
            finish(s, r, st, t_done);
        }
        s->cv_done.notify_all();
    }
}

// An admitted order of the streaming mode: the source slot of every pick and
// the rows it waits for.
struct Live {
    Request *r = nullptr;
    std::vector<uint32_t> slot;   // per pick: row * 64 + lane
    std::vector<uint32_t> rows;   // distinct rows
};

// Streaming mode; returns false (nothing admitted yet) if the state cannot
// be built, and then the caller falls back to step batching.
bool run_stream_mode(wr_server *s) {
    wr_graph *g = s->g;
    uint32_t want = (s->opts.max_source_slots + 63) / 64;
    try {
        const uint64_t per = stream_bytes_per_block(g);
        const uint64_t fit = s->budget > (8ull << 20) ? (s->budget - (8ull << 20)) / per : 0;
        want = static_cast<uint32_t>(std::min<uint64_t>(want, fit));
        if (!want) return false;
        s->stream = stream_create(g, want);
    } catch (const Error &) {
        return false;
    }
    const uint32_t R = stream_blocks(s->stream);
    std::vector<uint32_t> refcnt(R, 0);       // admitted orders using the row
    std::vector<uint8_t> busy(R, 0);          // row still relaxing
    std::vector<uint32_t> free_rows;
    for (uint32_t b = R; b-- > 0;) free_rows.push_back(b);
    std::vector<Live> live;
    std::vector<uint32_t> pending;
    std::vector<WeightBatch> ups;
    auto fail_all = [&](wr_status st) {
        std::unique_lock<std::mutex> lk(s->mu);
        const double t = clock_s();
        for (Live &L : live) finish(s, L.r, st, t);
        live.clear();
        s->cv_done.notify_all();
    };
    for (;;) {
        std::vector<Request *> adm;
        std::vector<uint32_t> rows, srcv;
        std::vector<Live> fresh;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const double tw0 = clock_s();
            if (live.empty())
                s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->updates.empty(); });
            s->t_wait += clock_s() - tw0;
            if (s->stop && s->queue.empty() && s->updates.empty() && live.empty()) return true;
            const bool update_waiting = !s->updates.empty();
            if (update_waiting && live.empty()) {
                while (!s->updates.empty()) {
                    ups.push_back(std::move(s->updates.front()));
                    s->updates.pop_front();
                }
            }
            if (!update_waiting) {
                // admission in arrival order while free rows last; the picks
                // of the orders admitted together share source lanes
                std::unordered_map<uint32_t, uint32_t> slot_of;
                std::vector<uint32_t> group;   // distinct picks of the group
                const double now = clock_s() - s->t0;
                while (!s->queue.empty()) {
                    Request *r = s->queue.front();
                    // distinct picks of the order, and those new to this group
                    std::unordered_map<uint32_t, uint32_t> seen;
                    uint32_t add = 0;
                    for (uint32_t v : r->picks)
                        if (seen.emplace(v, 0u).second && !slot_of.count(v)) ++add;
                    if ((seen.size() + 63) / 64 > R) {
                        // larger than the whole state: can never be admitted
                        s->queue.pop_front();
                        r->info.t_admit = now;
                        finish(s, r, WR_E_NOMEM, clock_s());
                        s->cv_done.notify_all();
                        continue;
                    }
                    if ((group.size() + add + 63) / 64 > free_rows.size()) break;
                    s->queue.pop_front();
                    for (uint32_t v : r->picks)
                        if (slot_of.emplace(v, 0u).second) group.push_back(v);
                    Live L;
                    L.r = r;
                    r->info.t_admit = now;
                    r->info.epoch = g->epoch;
                    fresh.push_back(std::move(L));
                }
                if (!group.empty()) {
                    // lanes in tile order: a row's sources start close together,
                    // so their wavefronts share tile visits
                    const std::vector<uint32_t> &tile_of = g->tiles->tile_of;
                    const std::vector<uint64_t> &tkey = tile_order_keys(g);
                    auto k = [&](uint32_t x) { return tile_of[x] == NONE ? ~0ull : tkey[tile_of[x]]; };
                    std::sort(group.begin(), group.end(), [&](uint32_t x, uint32_t y) {
                        if (k(x) != k(y)) return k(x) < k(y);
                        if (tile_of[x] != tile_of[y]) return tile_of[x] < tile_of[y];
                        return x < y;
                    });
                    const size_t nrows = (group.size() + 63) / 64;
                    for (size_t i = 0; i < nrows; ++i) {
                        rows.push_back(free_rows.back());
                        free_rows.pop_back();
                    }
                    srcv.assign(nrows * 64, NONE);
                    for (size_t k = 0; k < group.size(); ++k) {
                        srcv[k] = group[k];
                        slot_of[group[k]] = rows[k / 64] * 64 + static_cast<uint32_t>(k % 64);
                    }
                    for (Live &L : fresh) {
                        for (uint32_t v : L.r->picks) L.slot.push_back(slot_of[v]);
                        for (uint32_t sl : L.slot) L.rows.push_back(sl / 64);
                        std::sort(L.rows.begin(), L.rows.end());
                        L.rows.erase(std::unique(L.rows.begin(), L.rows.end()), L.rows.end());
                    }
                }
            }
        }
        if (!ups.empty()) {
            const double tu0 = clock_s();
            apply_updates(s, ups);
            s->t_update += clock_s() - tu0;
            // nothing is in flight; weights beyond the overlay tables' range
            // move serving to step batching
            try {
                (void)stream_bytes_per_block(g);
            } catch (const Error &) {
                stream_destroy(s->stream);
                s->stream = nullptr;
                run_step_mode(s);
                return true;
            }
        }
        bool admitted = fresh.empty();   // the orders taken from the queue are in flight
        try {
            if (!rows.empty()) {
                const double ta0 = clock_s();
                stream_admit(s->stream, rows, srcv);
                s->t_admit += clock_s() - ta0;
                s->rows_admitted += rows.size();
                for (uint32_t b : rows) busy[b] = 1;
                for (Live &L : fresh) {
                    for (uint32_t b : L.rows) ++refcnt[b];
                    live.push_back(std::move(L));
                }
            }
            admitted = true;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->max_inflight = std::max<uint32_t>(s->max_inflight, static_cast<uint32_t>(live.size()));
            }
            if (live.empty()) continue;
            const double ts0 = clock_s();
            stream_step(s->stream, pending);
            s->t_step += clock_s() - ts0;
            for (uint32_t b = 0; b < R; ++b)
                if (busy[b] && !pending[b]) busy[b] = 0;
            // retire the orders whose rows have all converged
            std::vector<uint32_t> off(1, 0u), picks, slots;
            std::vector<size_t> done;
            for (size_t i = 0; i < live.size(); ++i) {
                bool ok = true;
                for (uint32_t b : live[i].rows) ok = ok && !busy[b];
                if (!ok) continue;
                done.push_back(i);
                picks.insert(picks.end(), live[i].r->picks.begin(), live[i].r->picks.end());
                slots.insert(slots.end(), live[i].slot.begin(), live[i].slot.end());
                off.push_back(static_cast<uint32_t>(picks.size()));
            }
            {
                std::lock_guard<std::mutex> lk(s->mu);
                ++s->steps;
            }
            if (done.empty()) continue;
            uint64_t total = 0;
            for (size_t o = 0; o + 1 < off.size(); ++o)
                total += static_cast<uint64_t>(off[o + 1] - off[o]) * (off[o + 1] - off[o]);
            std::vector<uint32_t> out(total);
            const double tg0 = clock_s();
            stream_gather(s->stream, off, picks, slots, out.data());
            s->t_gather += clock_s() - tg0;
            const double t_done = clock_s();
            std::lock_guard<std::mutex> lk(s->mu);
            uint64_t at = 0;
            for (size_t k = 0; k < done.size(); ++k) {
                Live &L = live[done[k]];
                const uint64_t n = static_cast<uint64_t>(L.r->picks.size()) * L.r->picks.size();
                L.r->dist.assign(out.begin() + at, out.begin() + at + n);
                at += n;
                finish(s, L.r, WR_OK, t_done);
                for (uint32_t b : L.rows)
                    if (--refcnt[b] == 0) free_rows.push_back(b);
                L.r = nullptr;
            }
            live.erase(std::remove_if(live.begin(), live.end(), [](const Live &L) { return !L.r; }), live.end());
            s->cv_done.notify_all();
        } catch (const Error &e) {
            // a failed step fails the orders in flight (and those it was
            // admitting) and the state is built afresh; serving goes on (in
            // step batching if that fails too)
            set_last_error(e.msg);
            if (!admitted) {
                std::lock_guard<std::mutex> lk(s->mu);
                const double t = clock_s();
                for (Live &L : fresh) finish(s, L.r, e.st, t);
            }
            fail_all(e.st);
            std::fill(refcnt.begin(), refcnt.end(), 0u);
            std::fill(busy.begin(), busy.end(), 0);
            free_rows.clear();
            for (uint32_t b = R; b-- > 0;) free_rows.push_back(b);
            stream_destroy(s->stream);
            s->stream = nullptr;
            try {
                s->stream = stream_create(g, R);
            } catch (const Error &) {
                run_step_mode(s);
                return true;
            }
        }
    }
}

void scheduler(wr_server *s) {
    (void)hipSetDevice(s->g->ctx->device);
    if (!run_stream_mode(s)) run_step_mode(s);
}

Request *find(wr_server *s, uint64_t ticket) {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

wr_status wr_server_create(wr_graph *g, const wr_server_opts *opts, wr_server **out) {
    WR_API_BEGIN
    if (!g || !out) fail(WR_E_INVALID, "graph or out is NULL");
    *out = nullptr;
    auto s = std::make_unique<wr_server>();
    s->g = g;
    if (opts) s->opts = *opts;
    if (!s->opts.max_source_slots) s->opts.max_source_slots = 8192;
    if (!s->opts.max_queue) s->opts.max_queue = 65536;
    if (s->opts.passes_per_step) g->passes_per_replay = std::max(2u, s->opts.passes_per_step & ~1u);
    s->budget = s->opts.mem_budget_bytes ? s->opts.mem_budget_bytes : g->ctx->available();
    s->t0 = clock_s();
    wr_server *raw = s.get();
    s->worker = std::thread(scheduler, raw);
    *out = s.release();
    WR_API_END
}

wr_status wr_server_submit(wr_server *srv, uint32_t P, const uint32_t *picks, uint64_t *ticket) {
    WR_API_BEGIN
    if (!srv || !ticket) fail(WR_E_INVALID, "server or ticket is NULL");
    if (P > 0 && !picks) fail(WR_E_INVALID, "picks is NULL");
    for (uint32_t i = 0; i < P; ++i)
        if (picks[i] >= srv->g->V) fail(WR_E_INVALID, "pick out of range");
    auto r = std::make_unique<Request>();
    r->picks.assign(picks, picks + P);
    r->info.P = P;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) fail(WR_E_INVALID, "server is shutting down");
        if (srv->queue.size() >= srv->opts.max_queue) fail(WR_E_BUSY, "request queue is full");
        const double now = clock_s() - srv->t0;
        r->ticket = srv->next_ticket++;
        r->info.t_arrive = now;
        if (srv->first_arrive < 0) srv->first_arrive = now;
        ++srv->submitted;
        ++srv->outstanding;
        *ticket = r->ticket;
        Request *raw = r.release();
        srv->reqs[raw->ticket] = raw;
        if (P == 0) {
            // nothing to relax: done at once on the current epoch
            raw->info.t_admit = now;
            raw->info.epoch = srv->g->epoch;
            finish(srv, raw, WR_OK, clock_s());
            srv->cv_done.notify_all();
        } else {
            srv->queue.push_back(raw);
            srv->cv_work.notify_one();
        }
    }
    WR_API_END
}

wr_status wr_server_poll(wr_server *srv, uint64_t ticket, uint32_t *dist_out, wr_req_info *info) {
    WR_API_BEGIN
    if (!srv) fail(WR_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    Request *r = find(srv, ticket);
    if (!r) fail(WR_E_INVALID, "unknown or already collected ticket");
    if (!r->done) return WR_E_BUSY;
    if (info) *info = r->info;
    const wr_status st = r->info.status;
    if (st == WR_OK && !r->dist.empty()) {
        if (!dist_out) fail(WR_E_INVALID, "dist_out is NULL");
        std::memcpy(dist_out, r->dist.data(), r->dist.size() * sizeof(uint32_t));
    }
    srv->reqs.erase(ticket);
    delete r;
    if (st != WR_OK) fail(st, "request failed");
    WR_API_END
}

wr_status wr_server_update_weights(wr_server *srv, uint32_t n, const uint32_t *arc_index, const uint32_t *new_w) {
    WR_API_BEGIN
    if (!srv) fail(WR_E_INVALID, "server is NULL");
    if (n > 0 && (!arc_index || !new_w)) fail(WR_E_INVALID, "arc_index or new_w is NULL");
    for (uint32_t i = 0; i < n; ++i)
        if (arc_index[i] >= srv->g->E) fail(WR_E_INVALID, "arc index out of range");
    WeightBatch b;
    b.arc.assign(arc_index, arc_index + n);
    b.w.assign(new_w, new_w + n);
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->updates.push_back(std::move(b));
    srv->cv_work.notify_one();
    WR_API_END
}

wr_status wr_server_stats(wr_server *srv, wr_stats *out) {
    WR_API_BEGIN
    if (!srv || !out) fail(WR_E_INVALID, "server or out is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    wr_stats st{};
    st.submitted = srv->submitted;
    st.completed = srv->completed;
    st.failed = srv->failed;
    st.steps = srv->steps;
    st.max_inflight_requests = srv->max_inflight;
    if (!srv->lat_ms.empty()) {
        std::vector<double> v = srv->lat_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const double x = p * (v.size() - 1);
            const size_t i = static_cast<size_t>(x);
            const double f = x - i;
            return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
        };
        st.p50_ms = pct(0.50);
        st.p99_ms = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        st.mean_ms = sum / v.size();
        const double span = srv->last_done - srv->first_arrive;
        st.throughput_per_s = span > 0 ? srv->completed / span : 0.0;
    }
    *out = st;
    WR_API_END
}

wr_status wr_server_drain(wr_server *srv) {
    WR_API_BEGIN
    if (!srv) fail(WR_E_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
    WR_API_END
}

wr_status wr_server_destroy(wr_server *srv) {
    WR_API_BEGIN
    if (!srv) return WR_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    if (srv->stream) stream_destroy(srv->stream);
    if (std::getenv("WR_TRACE"))
        std::fprintf(stderr,
                     "[wroute server] steps %llu rows admitted %llu | seconds: update %.3f admit %.3f "
                     "step %.3f gather %.3f idle %.3f\n",
                     static_cast<unsigned long long>(srv->steps), static_cast<unsigned long long>(srv->rows_admitted),
                     srv->t_update, srv->t_admit, srv->t_step, srv->t_gather, srv->t_wait);
    for (auto &kv : srv->reqs) delete kv.second;
    delete srv;
    WR_API_END
}

}  // extern "C"
