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
// Weight updates queue.  The streaming mode keeps two resident copies of the
// graph, each with its own rows: an update is applied to the copy whose rows
// have all retired, which then takes the new orders while the other copy's
// orders finish on their own epoch; step batching (and streaming when the
// copy cannot be made) applies updates once nothing is in flight.  Every
// order is solved entirely on the epoch current at its admission.  An
// order's matrix is the same alone or in any mix, because every schedule
// reaches the exact fixpoint.
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
    std::condition_variable cv_done;  // drain / poll waiters, and the scheduler's set-up
    bool ready = false;               // the scheduler has built its state
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
    uint64_t epoch_now = 0;           // epoch new orders are admitted on (streaming mode)
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

// The scheduler's state is built: wr_server_create may return.
void set_ready(wr_server *s) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->ready = true;
    s->cv_done.notify_all();
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
    set_ready(s);
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
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->epoch_now = s->g->epoch;
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

// One resident copy of the graph at one weight epoch, with its own block
// rows.  The streaming mode keeps two: new orders are admitted into the
// current one, and a weight update is applied to the other as soon as its
// rows have all retired, which then becomes current; the orders still in
// flight on the old copy finish on their own epoch.
struct Side {
    wr_graph *g = nullptr;
    bool owned = false;               // the server's own copy
    StreamSolver *stream = nullptr;
    uint64_t epoch = 0;               // server epoch of its weights
    std::vector<WeightBatch> lag;     // applied to the other copy, not yet here
    std::vector<uint32_t> refcnt;     // admitted orders using each row
    std::vector<uint8_t> busy;        // row still relaxing
    std::vector<uint32_t> free_rows;
    std::vector<Live> live;
    std::vector<uint32_t> pending;

    void reset_rows(uint32_t R) {
        refcnt.assign(R, 0u);
        busy.assign(R, 0);
        free_rows.clear();
        for (uint32_t b = R; b-- > 0;) free_rows.push_back(b);
    }
};

// A copy of g at its current weights: the same CSR, segmentation and
// schedule (schedule first: the tiles are sized by it).
wr_graph *clone_graph(wr_graph *g) {
    wr_graph *c = nullptr;
    wr_status st = wr_graph_create_csr(g->ctx, g->V, g->E, g->row_ptr.data(), g->col.data(), g->w.data(), 0, &c);
    if (st != WR_OK) fail(st, std::string("copying the graph: ") + wr_last_error());
    c->tile_vertices = g->tile_vertices;
    c->waves_per_group = g->waves_per_group;
    c->lanes = g->lanes;
    c->sources_per_unit = g->sources_per_unit;
    c->passes_per_replay = g->passes_per_replay;
    if (g->grid_W)
        st = wr_graph_segment_grid(c, g->grid_W, g->grid_H, g->grid_L, g->grid_tw, g->grid_th);
    else if (g->tiles_user)
        st = wr_graph_set_segments(c, g->user_seg.data(), g->user_num_segments);
    if (st != WR_OK) {
        const std::string msg = wr_last_error();
        wr_graph_destroy(c);
        fail(st, "segmenting the graph's copy: " + msg);
    }
    return c;
}

// Applies update batches to one copy; returns those it accepted (a batch the
// graph refuses is dropped, and would be refused by the other copy too).
std::vector<WeightBatch> apply_to(wr_graph *g, std::vector<WeightBatch> &ups) {
    std::vector<WeightBatch> ok;
    for (WeightBatch &u : ups) {
        uint64_t ep = 0;
        const wr_status st =
            wr_graph_update_weights(g, static_cast<uint32_t>(u.arc.size()), u.arc.data(), u.w.data(), &ep);
        if (st != WR_OK)
            set_last_error(std::string("server weight update rejected: ") + wr_status_str(st));
        else
            ok.push_back(std::move(u));
    }
    ups.clear();
    return ok;
}

// Streaming mode; returns false (nothing admitted yet) if the state cannot
// be built, and then the caller falls back to step batching.
bool run_stream_mode(wr_server *s) {
    wr_graph *g = s->g;
    uint32_t want = (s->opts.max_source_slots + 63) / 64;
    Side S[2];
    S[0].g = g;
    S[0].epoch = g->epoch;
    const bool two = s->opts.resident_epochs >= 2;
    try {
        const uint64_t per = stream_bytes_per_block(g);
        // rows for each copy's state (besides the second copy's graph and tables)
        const uint64_t fit = s->budget > (8ull << 20) ? (s->budget - (8ull << 20)) / ((two ? 2 : 1) * per) : 0;
        want = static_cast<uint32_t>(std::min<uint64_t>(want, fit));
        if (!want) return false;
        S[0].stream = stream_create(g, want);
    } catch (const Error &) {
        return false;   // step batching signals ready
    }
    const uint32_t R = stream_blocks(S[0].stream);
    S[0].reset_rows(R);
    // the second copy is made before serving starts; without it updates
    // wait for the rows in flight, as with one copy
    if (two) try {
        S[1].g = clone_graph(g);
        S[1].owned = true;
        S[1].epoch = S[0].epoch;
        S[1].stream = stream_create(S[1].g, R);
        S[1].reset_rows(R);
    } catch (...) {
        set_last_error("no second copy of the graph: weight updates wait for the orders in flight");
        if (S[1].stream) stream_destroy(S[1].stream);
        S[1].stream = nullptr;
        if (S[1].g) wr_graph_destroy(S[1].g);
        S[1].g = nullptr;
        S[1].owned = false;
    }
    set_ready(s);
    uint32_t cur = 0;
    std::vector<WeightBatch> waiting;   // updates taken from the queue, not applied yet
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->epoch_now = S[0].epoch;
    }
    auto fail_side = [&](Side &d, wr_status st) {
        std::unique_lock<std::mutex> lk(s->mu);
        const double t = clock_s();
        for (Live &L : d.live) finish(s, L.r, st, t);
        d.live.clear();
        s->cv_done.notify_all();
    };
    // the caller's graph ends at the newest accepted weights
    auto catch_up_caller = [&]() {
        if (!S[0].lag.empty()) {
            (void)apply_to(S[0].g, S[0].lag);
            S[0].lag.clear();
        }
    };
    // steps one copy's rows once and retires its converged orders
    auto step_side = [&](Side &d) {
        const double ts0 = clock_s();
        stream_step(d.stream, d.pending);
        s->t_step += clock_s() - ts0;
        for (uint32_t b = 0; b < R; ++b)
            if (d.busy[b] && !d.pending[b]) d.busy[b] = 0;
        std::vector<uint32_t> off(1, 0u), picks, slots;
        std::vector<size_t> done;
        for (size_t i = 0; i < d.live.size(); ++i) {
            bool ok = true;
            for (uint32_t b : d.live[i].rows) ok = ok && !d.busy[b];
            if (!ok) continue;
            done.push_back(i);
            picks.insert(picks.end(), d.live[i].r->picks.begin(), d.live[i].r->picks.end());
            slots.insert(slots.end(), d.live[i].slot.begin(), d.live[i].slot.end());
            off.push_back(static_cast<uint32_t>(picks.size()));
        }
        if (done.empty()) return;
        uint64_t total = 0;
        for (size_t o = 0; o + 1 < off.size(); ++o)
            total += static_cast<uint64_t>(off[o + 1] - off[o]) * (off[o + 1] - off[o]);
        std::vector<uint32_t> out(total);
        const double tg0 = clock_s();
        stream_gather(d.stream, off, picks, slots, out.data());
        s->t_gather += clock_s() - tg0;
        const double t_done = clock_s();
        std::lock_guard<std::mutex> lk(s->mu);
        uint64_t at = 0;
        for (size_t k = 0; k < done.size(); ++k) {
            Live &L = d.live[done[k]];
            const uint64_t n = static_cast<uint64_t>(L.r->picks.size()) * L.r->picks.size();
            L.r->dist.assign(out.begin() + at, out.begin() + at + n);
            at += n;
            finish(s, L.r, WR_OK, t_done);
            for (uint32_t b : L.rows)
                if (--d.refcnt[b] == 0) d.free_rows.push_back(b);
            L.r = nullptr;
        }
        d.live.erase(std::remove_if(d.live.begin(), d.live.end(), [](const Live &L) { return !L.r; }),
                     d.live.end());
        s->cv_done.notify_all();
    };
    // serving moves to step batching on the caller's graph (weights beyond
    // the overlay tables' range): the other copy's orders finish first
    auto to_step_mode = [&](uint32_t bad) {
        Side &o = S[1 - bad];
        while (o.stream && !o.live.empty()) step_side(o);
        for (Side &d : S) {
            if (d.stream) stream_destroy(d.stream);
            d.stream = nullptr;
        }
        catch_up_caller();
        if (S[1].owned) wr_graph_destroy(S[1].g);
        S[1].g = nullptr;
        run_step_mode(s);
        return true;
    };
    for (;;) {
        Side &C = S[cur];
        std::vector<Live> fresh;
        std::vector<uint32_t> rows, srcv;
        bool admitting = true;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const double tw0 = clock_s();
            if (S[0].live.empty() && S[1].live.empty() && waiting.empty())
                s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty() || !s->updates.empty(); });
            s->t_wait += clock_s() - tw0;
            if (s->stop && s->queue.empty() && s->updates.empty() && waiting.empty() && S[0].live.empty() &&
                S[1].live.empty()) {
                lk.unlock();
                for (Side &d : S) {
                    if (d.stream) stream_destroy(d.stream);
                    d.stream = nullptr;
                }
                catch_up_caller();
                if (S[1].owned) wr_graph_destroy(S[1].g);
                S[1].g = nullptr;
                return true;
            }
            while (!s->updates.empty()) {
                waiting.push_back(std::move(s->updates.front()));
                s->updates.pop_front();
            }
        }
        // ---- weight updates: onto the copy with nothing in flight
        if (!waiting.empty()) {
            const uint32_t o = 1 - cur;
            const double tu0 = clock_s();
            uint32_t target = NONE;
            if (S[o].g && S[o].live.empty())
                target = o;
            else if (!S[o].g && C.live.empty())
                target = cur;
            if (target != NONE) {
                Side &T = S[target];
                std::vector<WeightBatch> todo = std::move(T.lag);
                T.lag.clear();
                const size_t nlag = todo.size();
                for (WeightBatch &u : waiting) todo.push_back(std::move(u));
                waiting.clear();
                std::vector<WeightBatch> ok = apply_to(T.g, todo);
                // the lag had been accepted before; the new batches count
                const uint64_t fresh_n = ok.size() >= nlag ? ok.size() - nlag : 0;
                if (target != cur) {
                    for (size_t k = nlag; k < ok.size(); ++k) S[cur].lag.push_back(ok[k]);
                    T.epoch = C.epoch + fresh_n;
                    if (fresh_n) cur = target;
                } else {
                    T.epoch += fresh_n;
                }
                s->t_update += clock_s() - tu0;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    s->epoch_now = S[cur].epoch;
                }
                try {
                    (void)stream_bytes_per_block(T.g);
                } catch (const Error &) {
                    return to_step_mode(target);
                }
            } else if (!S[o].g) {
                admitting = false;   // one copy: admission waits for the rows in flight
            }
        }
        Side &A = S[cur];
        // ---- admission in arrival order while free rows last; the picks of
        // the orders admitted together share source lanes
        if (admitting) {
            std::unique_lock<std::mutex> lk(s->mu);
            std::unordered_map<uint32_t, uint32_t> slot_of;
            std::vector<uint32_t> group;   // distinct picks of the group
            const double now = clock_s() - s->t0;
            while (!s->queue.empty()) {
                Request *r = s->queue.front();
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
                if ((group.size() + add + 63) / 64 > A.free_rows.size()) break;
                s->queue.pop_front();
                for (uint32_t v : r->picks)
                    if (slot_of.emplace(v, 0u).second) group.push_back(v);
                Live L;
                L.r = r;
                r->info.t_admit = now;
                r->info.epoch = A.epoch;
                fresh.push_back(std::move(L));
            }
            if (!group.empty()) {
                // lanes in tile order: a row's sources start close together,
                // so their wavefronts share tile visits
                const std::vector<uint32_t> &tile_of = A.g->tiles->tile_of;
                const std::vector<uint64_t> &tkey = tile_order_keys(A.g);
                auto k = [&](uint32_t x) { return tile_of[x] == NONE ? ~0ull : tkey[tile_of[x]]; };
                std::sort(group.begin(), group.end(), [&](uint32_t x, uint32_t y) {
                    if (k(x) != k(y)) return k(x) < k(y);
                    if (tile_of[x] != tile_of[y]) return tile_of[x] < tile_of[y];
                    return x < y;
                });
                const size_t nrows = (group.size() + 63) / 64;
                for (size_t i = 0; i < nrows; ++i) {
                    rows.push_back(A.free_rows.back());
                    A.free_rows.pop_back();
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
        bool admitted = fresh.empty();   // the orders taken from the queue are in flight
        uint32_t stepping = cur;
        try {
            if (!rows.empty()) {
                const double ta0 = clock_s();
                stream_admit(A.stream, rows, srcv);
                s->t_admit += clock_s() - ta0;
                s->rows_admitted += rows.size();
                for (uint32_t b : rows) A.busy[b] = 1;
                for (Live &L : fresh) {
                    for (uint32_t b : L.rows) ++A.refcnt[b];
                    A.live.push_back(std::move(L));
                }
            }
            admitted = true;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->max_inflight = std::max<uint32_t>(
                    s->max_inflight, static_cast<uint32_t>(S[0].live.size() + S[1].live.size()));
            }
            // one step of each copy with rows in flight, the older epoch first
            bool stepped = false;
            for (uint32_t k = 0; k < 2; ++k) {
                stepping = (cur + 1 + k) % 2;
                if (S[stepping].stream && !S[stepping].live.empty()) {
                    step_side(S[stepping]);
                    stepped = true;
                }
            }
            if (stepped) {
                std::lock_guard<std::mutex> lk(s->mu);
                ++s->steps;
            }
        } catch (const Error &e) {
            // a failed step fails the orders in flight on that copy (and those
            // being admitted), and its state is built afresh; serving goes on
            // (in step batching if that fails too)
            set_last_error(e.msg);
            if (!admitted) {
                std::lock_guard<std::mutex> lk(s->mu);
                const double t = clock_s();
                for (Live &L : fresh) finish(s, L.r, e.st, t);
                stepping = cur;
            }
            Side &d = S[stepping];
            fail_side(d, e.st);
            d.reset_rows(R);
            stream_destroy(d.stream);
            d.stream = nullptr;
            try {
                d.stream = stream_create(d.g, R);
            } catch (const Error &) {
                if (stepping == 0 && !S[1].g) return to_step_mode(0);
                // serve on the other copy alone, or on the caller's graph
                fail_side(S[1 - stepping], e.st);
                return to_step_mode(stepping);
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
    if (s->opts.resident_epochs > 2) fail(WR_E_INVALID, "resident_epochs must be 0, 1 or 2");
    s->budget = s->opts.mem_budget_bytes ? s->opts.mem_budget_bytes : g->ctx->available();
    s->epoch_now = g->epoch;
    s->t0 = clock_s();
    wr_server *raw = s.get();
    s->worker = std::thread(scheduler, raw);
    {
        // serving starts once the scheduler has built its state
        std::unique_lock<std::mutex> lk(raw->mu);
        raw->cv_done.wait(lk, [&] { return raw->ready; });
    }
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
            raw->info.epoch = srv->epoch_now;
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
