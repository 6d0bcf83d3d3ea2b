// Host runtime: status strings, thread-local errors, fault injection, the
// device context with its memory budget, graph residency, CSR validation and
// weight epochs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <mutex>
#include <numeric>

#include "wr_internal.hpp"

namespace wr {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }

[[noreturn]] void fail(wr_status st, const std::string &msg) { throw Error{st, msg}; }

// ------------------------------------------------------------ fault hooks
// Test hooks: the n-th next device allocation (kind 1) or kernel launch
// (kind 2) the library makes fails on the host with the status a real
// failure of that call would give, before anything reaches the device.
// Armed by wr_debug_fault, or at start-up by WR_FAULT=alloc:N | launch:N.
namespace {
std::atomic<uint32_t> g_fault_kind{0};
std::atomic<long> g_fault_left{0};
struct FaultEnv {
    FaultEnv() {
        const char *e = std::getenv("WR_FAULT");
        if (!e) return;
        std::string s(e);
        size_t c = s.find(':');
        if (c == std::string::npos) return;
        const long n = std::atol(s.c_str() + c + 1);
        if (n <= 0) return;
        if (s.compare(0, c, "alloc") == 0) g_fault_kind = 1;
        if (s.compare(0, c, "launch") == 0) g_fault_kind = 2;
        g_fault_left = n;
    }
} g_fault_env;
bool fault_now(uint32_t kind) {
    if (g_fault_kind.load() != kind) return false;
    if (--g_fault_left != 0) return false;
    g_fault_kind = 0;
    return true;
}
}  // namespace

bool fault_alloc_now() { return fault_now(1); }
bool fault_launch_now() { return fault_now(2); }

void check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(WR_E_DEVICE, std::string("launch ") + what + ": " + hipGetErrorString(e));
}

}  // namespace wr

using namespace wr;

// ---------------------------------------------------------------- context
void *wr_context::alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    if (used.load() + bytes > budget)
        fail(WR_E_NOMEM, "device budget exceeded: need " + std::to_string(bytes) + " more bytes, " +
                             std::to_string(available()) + " available");
    if (fault_alloc_now()) fail(WR_E_NOMEM, "injected allocation failure");
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        fail(WR_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes: out of memory");
    }
    if (e != hipSuccess) fail(WR_E_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    used += bytes;
    return p;
}

void wr_context::release(void *p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    used -= bytes;
}

wr_graph::~wr_graph() {
    destroy_workspace(ws);
    delete tiles;
}

extern "C" {

const char *wr_status_str(wr_status s) {
    switch (s) {
    case WR_OK: return "WR_OK";
    case WR_E_INVALID: return "WR_E_INVALID";
    case WR_E_RANGE: return "WR_E_RANGE";
    case WR_E_NOMEM: return "WR_E_NOMEM";
    case WR_E_DEVICE: return "WR_E_DEVICE";
    case WR_E_UNSUPPORTED: return "WR_E_UNSUPPORTED";
    case WR_E_BUSY: return "WR_E_BUSY";
    case WR_E_INTERNAL: return "WR_E_INTERNAL";
    }
    return "WR_E_UNKNOWN";
}

const char *wr_last_error(void) { return g_last_error.c_str(); }

const char *wr_version(void) { return "wroute 0.1.0 (gfx950)"; }

wr_status wr_context_create(int device, uint64_t mem_budget_bytes, wr_context **out) {
    WR_API_BEGIN
    if (!out) fail(WR_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) fail(WR_E_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) fail(WR_E_INVALID, "device index out of range");
    WR_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    WR_HIP(hipGetDeviceProperties(&prop, device));
    auto *ctx = new wr_context();
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;
    size_t freeb = 0, totalb = 0;
    WR_HIP(hipMemGetInfo(&freeb, &totalb));
    ctx->budget = mem_budget_bytes ? mem_budget_bytes : static_cast<uint64_t>(freeb * 0.9);
    hipError_t se = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    if (se == hipSuccess) se = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    if (se != hipSuccess) {
        if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        fail(WR_E_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(se));
    }
    *out = ctx;
    WR_API_END
}

wr_status wr_context_destroy(wr_context *ctx) {
    WR_API_BEGIN
    if (!ctx) return WR_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    WR_API_END
}

wr_status wr_context_memory(const wr_context *ctx, uint64_t *used, uint64_t *budget) {
    WR_API_BEGIN
    if (!ctx) fail(WR_E_INVALID, "ctx is NULL");
    if (used) *used = ctx->used.load();
    if (budget) *budget = ctx->budget;
    WR_API_END
}

}  // extern "C"

// --------------------------------------------------------------- validation
namespace {

// Structure checks; returns the number of vertices incident to an arc and the
// maximum weight through the out-parameters.
void validate_structure(uint32_t V, uint32_t E, const uint32_t *row_ptr, const uint32_t *col,
                        const uint32_t *w, uint32_t *n_inc, uint32_t *max_w, uint64_t *zero_w) {
    if (!row_ptr) fail(WR_E_INVALID, "row_ptr is NULL");
    if (E > 0 && (!col || !w)) fail(WR_E_INVALID, "col or w is NULL");
    if (V == 0) fail(WR_E_INVALID, "V must be positive");
    if (V >= 0x80000000u) fail(WR_E_INVALID, "V must be below 2^31");
    if (row_ptr[0] != 0) fail(WR_E_INVALID, "row_ptr[0] must be 0");
    if (row_ptr[V] != E) fail(WR_E_INVALID, "row_ptr[V] must equal E");
    for (uint32_t v = 0; v < V; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) fail(WR_E_INVALID, "row_ptr must be non-decreasing");
    std::vector<uint8_t> inc(V, 0);
    uint32_t mw = 0;
    uint64_t zw = 0;
    for (uint32_t u = 0; u < V; ++u) {
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            if (col[e] >= V) fail(WR_E_INVALID, "col[" + std::to_string(e) + "] out of range");
            inc[u] = 1;
            inc[col[e]] = 1;
            mw = std::max(mw, w[e]);
            zw += w[e] == 0;
        }
    }
    uint32_t ni = 0;
    for (uint32_t v = 0; v < V; ++v) ni += inc[v];
    if (ni > 1 && static_cast<uint64_t>(mw) * (ni - 1) >= static_cast<uint64_t>(INF))
        fail(WR_E_RANGE, "max weight times (incident vertices - 1) reaches WR_INF");
    *n_inc = ni;
    *max_w = mw;
    *zero_w = zw;
}

}  // namespace

extern "C" {

wr_status wr_validate_csr(uint32_t V, uint32_t E, const uint32_t *row_ptr, const uint32_t *col,
                          const uint32_t *w) {
    WR_API_BEGIN
    uint32_t ni, mw;
    uint64_t zw;
    validate_structure(V, E, row_ptr, col, w, &ni, &mw, &zw);
    WR_API_END
}

wr_status wr_graph_create_csr(wr_context *ctx, uint32_t V, uint32_t E, const uint32_t *row_ptr,
                              const uint32_t *col, const uint32_t *w, uint32_t flags,
                              wr_graph **out) {
    WR_API_BEGIN
    if (!ctx || !out) fail(WR_E_INVALID, "ctx or out is NULL");
    (void)flags;
    *out = nullptr;
    uint32_t ni, mw;
    uint64_t zw;
    validate_structure(V, E, row_ptr, col, w, &ni, &mw, &zw);
    WR_HIP(hipSetDevice(ctx->device));
    auto *g = new wr_graph();
    try {
        g->ctx = ctx;
        g->V = V;
        g->E = E;
        g->n_incident = ni;
        g->max_w = mw;
        g->zero_w = zw;
        g->row_ptr.assign(row_ptr, row_ptr + V + 1);
        g->col.assign(col, col + E);
        g->w.assign(w, w + E);
        // in-arc CSR (transpose) for pull sweeps and predecessors
        std::vector<uint32_t> in_ptr(V + 1, 0), in_src(E), in_w(E);
        g->in_pos_of_arc.resize(E);
        for (uint32_t e = 0; e < E; ++e) in_ptr[col[e] + 1]++;
        for (uint32_t v = 0; v < V; ++v) in_ptr[v + 1] += in_ptr[v];
        std::vector<uint32_t> fill(in_ptr.begin(), in_ptr.end() - 1);
        for (uint32_t u = 0; u < V; ++u)
            for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                const uint32_t p = fill[col[e]]++;
                in_src[p] = u;
                in_w[p] = w[e];
                g->in_pos_of_arc[e] = p;
            }
        hipStream_t st = ctx->stream;
        upload(g->d_row_ptr, ctx, g->row_ptr, st);
        upload(g->d_col, ctx, g->col, st);
        upload(g->d_w, ctx, g->w, st);
        upload(g->d_in_ptr, ctx, in_ptr, st);
        upload(g->d_in_src, ctx, in_src, st);
        upload(g->d_in_w, ctx, in_w, st);
        upload(g->d_in_pos_of_arc, ctx, g->in_pos_of_arc, st);
        WR_HIP(hipStreamSynchronize(st));
    } catch (...) {
        delete g;
        throw;
    }
    *out = g;
    WR_API_END
}

wr_status wr_graph_destroy(wr_graph *g) {
    WR_API_BEGIN
    if (!g) return WR_OK;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    delete g;
    WR_API_END
}

wr_status wr_graph_epoch(const wr_graph *g, uint64_t *epoch) {
    WR_API_BEGIN
    if (!g || !epoch) fail(WR_E_INVALID, "NULL argument");
    *epoch = g->epoch;
    WR_API_END
}

wr_status wr_graph_update_weights(wr_graph *g, uint32_t n, const uint32_t *arc_index,
                                  const uint32_t *new_w, uint64_t *out_epoch) {
    WR_API_BEGIN
    if (!g) fail(WR_E_INVALID, "graph is NULL");
    if (n > 0 && (!arc_index || !new_w)) fail(WR_E_INVALID, "NULL update arrays");
    for (uint32_t i = 0; i < n; ++i)
        if (arc_index[i] >= g->E) fail(WR_E_INVALID, "arc index out of range");
    // last entry for an arc wins: keep the final value per arc
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return arc_index[a] < arc_index[b]; });
    std::vector<uint32_t> arcs, vals;
    arcs.reserve(n);
    vals.reserve(n);
    for (uint32_t k = 0; k < n; ++k) {
        const uint32_t i = order[k];
        if (k + 1 < n && arc_index[order[k + 1]] == arc_index[i]) continue;
        arcs.push_back(arc_index[i]);
        vals.push_back(new_w[i]);
    }
    // apply on the host mirror; undo if the overflow bound would break
    std::vector<uint32_t> old(arcs.size());
    uint32_t mw = g->max_w;
    bool rescan = false;
    int64_t dz = 0;
    for (size_t k = 0; k < arcs.size(); ++k) {
        old[k] = g->w[arcs[k]];
        if (vals[k] > mw) mw = vals[k];
        if (old[k] == g->max_w && vals[k] < old[k]) rescan = true;
        dz += (vals[k] == 0) - (old[k] == 0);
        g->w[arcs[k]] = vals[k];
    }
    if (rescan) {
        mw = 0;
        for (uint32_t x : g->w) mw = std::max(mw, x);
    }
    if (g->n_incident > 1 && static_cast<uint64_t>(mw) * (g->n_incident - 1) >= INF) {
        for (size_t k = 0; k < arcs.size(); ++k) g->w[arcs[k]] = old[k];
        fail(WR_E_RANGE, "updated weights break the overflow bound");
    }
    g->max_w = mw;
    g->zero_w = static_cast<uint64_t>(static_cast<int64_t>(g->zero_w) + dz);
    wr_context *ctx = g->ctx;
    WR_HIP(hipSetDevice(ctx->device));
    if (!arcs.empty()) {
        DBuf<uint32_t> da, dv;
        upload(da, ctx, arcs, ctx->stream);
        upload(dv, ctx, vals, ctx->stream);
        TileSet *ts = g->tiles;
        launch_weight_scatter(static_cast<uint32_t>(arcs.size()), da.p, dv.p, g->d_w.p, g->d_in_w.p,
                              g->d_in_pos_of_arc.p, ts ? ts->d_l_arc.p : nullptr,
                              ts ? ts->d_x_w.p : nullptr, ts ? ts->d_arc_slot.p : nullptr,
                              ts ? ts->d_li_arc.p : nullptr, ts ? ts->d_arc_slot_in.p : nullptr,
                              ctx->stream);
        if (ts) {
            for (size_t k = 0; k < arcs.size(); ++k) {
                const uint32_t sl = ts->arc_slot[arcs[k]];
                if (sl & 0x80000000u)
                    ts->x_w[sl & 0x7FFFFFFFu] = vals[k];
                else
                    ts->l_arc[sl] = (ts->l_arc[sl] & 0xFFFF0000u) | (vals[k] & 0xFFFFu);
                const uint32_t si = ts->arc_slot_in[arcs[k]];
                if (si != NONE) ts->li_arc[si] = (ts->li_arc[si] & 0xFFFF0000u) | (vals[k] & 0xFFFFu);
            }
        }
        WR_HIP(hipStreamSynchronize(ctx->stream));
    }
    g->epoch += 1;
    if (out_epoch) *out_epoch = g->epoch;
    WR_API_END
}

}  // extern "C"

extern "C" wr_status wr_debug_fault(uint32_t kind, uint64_t nth) {
    WR_API_BEGIN
    if (kind > 2) fail(WR_E_INVALID, "fault kind must be 0 (off), 1 (allocation) or 2 (launch)");
    if (kind != 0 && nth == 0) fail(WR_E_INVALID, "nth must be positive");
    g_fault_kind = 0;
    g_fault_left = static_cast<long>(nth);
    g_fault_kind = kind;
    WR_API_END
}
