// Continuous-batching server: orders arrive at any time, a scheduler thread
// admits as many queued orders as the source slots and the memory budget
// allow, solves the admitted batch in one multi-source call (distinct picks
// relaxed once, 64 sources per block), hands every order its P x P matrix,
// and admits the next batch.  Weight updates queue and are applied between
// steps, so each admitted order is solved entirely on one weight epoch (the
// epoch current at its admission), and an order's matrix is the same alone
// or in any mix, because every schedule reaches the exact fixpoint.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
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
};

namespace {

// Device bytes one admitted batch needs besides the graph: the output
// matrices plus the per-source relaxation state (rounded up to blocks of 64).
uint64_t batch_bytes(const wr_graph *g, uint64_t sources, uint64_t out_entries) {
    const TileSet *ts = g->tiles;
    const uint64_t blocks = (sources + 63) / 64;
    uint64_t per_block;
    if (ts)
        per_block = SegBuffers::bytes_per_row(*ts, 4, 64);
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

void scheduler(wr_server *s) {
    (void)hipSetDevice(s->g->ctx->device);
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
        for (WeightBatch &u : ups) {
            uint64_t ep = 0;
            const wr_status st = wr_graph_update_weights(s->g, static_cast<uint32_t>(u.arc.size()), u.arc.data(),
                                                         u.w.data(), &ep);
            if (st != WR_OK) set_last_error(std::string("server weight update rejected: ") + wr_status_str(st));
        }
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
        // one step: every admitted order in one call
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
    for (auto &kv : srv->reqs) delete kv.second;
    delete srv;
    WR_API_END
}

}  // extern "C"
