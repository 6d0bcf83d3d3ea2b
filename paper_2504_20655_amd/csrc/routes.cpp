// wr_order_routes: the optimal open route over each order's stops, from the
// order's distance matrix (Route Optimization section; Held and Karp's
// subset programme, run by k_route_hk with one workgroup per order).
#include <algorithm>
#include <mutex>
#include <vector>

#include "wr_internal.hpp"

using namespace wr;

namespace {

// Validated shape of a batch of orders: per-order matrix offsets, the total
// of matrix cells and of picks, and the largest order.
struct RouteBatch {
    std::vector<uint32_t> off;
    std::vector<uint64_t> mbase;
    uint64_t cells = 0;
    uint32_t total = 0, nmax = 0;
};

RouteBatch route_batch(uint32_t num_orders, const uint32_t *pick_offsets, uint32_t max_stops, const char *what) {
    if (!pick_offsets) fail(WR_E_INVALID, "pick_offsets is NULL");
    if (pick_offsets[0] != 0) fail(WR_E_INVALID, "pick_offsets[0] must be 0");
    RouteBatch b;
    b.mbase.resize(num_orders);
    for (uint32_t o = 0; o < num_orders; ++o) {
        if (pick_offsets[o + 1] < pick_offsets[o]) fail(WR_E_INVALID, "pick_offsets must be non-decreasing");
        const uint32_t P = pick_offsets[o + 1] - pick_offsets[o];
        if (P > max_stops)
            fail(WR_E_UNSUPPORTED, "order " + std::to_string(o) + " has " + std::to_string(P) + " stops; " + what +
                                       " are served for at most " + std::to_string(max_stops));
        b.mbase[o] = b.cells;
        b.cells += static_cast<uint64_t>(P) * P;
        b.nmax = std::max(b.nmax, P);
    }
    b.off.assign(pick_offsets, pick_offsets + num_orders + 1);
    b.total = pick_offsets[num_orders];
    return b;
}

// With caller (device) buffers, the library stream starts after the work the
// caller queued on `stream`.
void join_caller_stream(wr_context *ctx, bool dev, void *stream) {
    if (!dev) return;
    hipEvent_t ev;
    WR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    WR_HIP(hipEventRecord(ev, static_cast<hipStream_t>(stream)));
    WR_HIP(hipStreamWaitEvent(ctx->stream, ev, 0));
    (void)hipEventDestroy(ev);
}

}  // namespace

extern "C" wr_status wr_order_routes(wr_context *ctx, uint32_t num_orders, const uint32_t *pick_offsets,
                                     const uint32_t *dist, uint64_t *length_out, uint32_t *route_out,
                                     uint32_t flags, void *stream) {
    WR_API_BEGIN
    if (!ctx) fail(WR_E_INVALID, "context is NULL");
    if (flags & ~static_cast<uint32_t>(WR_DEVICE_PTRS | WR_ROUTE_ENUMERATE))
        fail(WR_E_INVALID, "unknown flags for wr_order_routes");
    if (num_orders == 0) return WR_OK;
    const bool enumerate = flags & WR_ROUTE_ENUMERATE;
    const RouteBatch rb = route_batch(num_orders, pick_offsets,
                                      enumerate ? route_enumerate_max_stops() : route_max_stops(),
                                      enumerate ? "enumerated routes" : "exact routes");
    const uint64_t cells = rb.cells;
    const uint32_t total = rb.total, nmax = rb.nmax;
    if (!length_out) fail(WR_E_INVALID, "length_out is NULL");
    if (total && !route_out) fail(WR_E_INVALID, "route_out is NULL");
    if (cells && !dist) fail(WR_E_INVALID, "dist is NULL");
    const bool dev = flags & WR_DEVICE_PTRS;
    WR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    join_caller_stream(ctx, dev, stream);
    DBuf<uint32_t> d_off, d_flag, d_dist, d_route;
    DBuf<uint64_t> d_base, d_len;
    upload(d_off, ctx, rb.off, st);
    upload(d_base, ctx, rb.mbase, st);
    d_flag.alloc(ctx, 1);
    launch_fill_u32(d_flag.p, 1, 0u, st);
    const uint32_t *ddist = dist;
    uint64_t *dlen = length_out;
    uint32_t *droute = route_out;
    if (!dev) {
        d_dist.alloc(ctx, std::max<uint64_t>(cells, 1));
        if (cells) WR_HIP(hipMemcpyAsync(d_dist.p, dist, cells * 4, hipMemcpyHostToDevice, st));
        d_len.alloc(ctx, num_orders);
        d_route.alloc(ctx, std::max(total, 1u));
        ddist = d_dist.p;
        dlen = d_len.p;
        droute = d_route.p;
    }
    DBuf<uint64_t> d_key;
    if (enumerate) {
        d_key.alloc(ctx, num_orders);
        launch_fill_u32(reinterpret_cast<uint32_t *>(d_key.p), 2ull * num_orders, 0xFFFFFFFFu, st);
        launch_route_perm(num_orders, d_off.p, d_base.p, ddist, reinterpret_cast<unsigned long long *>(d_key.p),
                          dlen, droute, d_flag.p, nmax, st);
    } else {
        // the LDS of the largest order bounds the workgroups per CU
        const uint32_t lds = route_lds_bytes(std::max(nmax, 1u));
        const uint32_t per_cu = std::max(1u, std::min(8u, (160u * 1024u) / lds));
        launch_route_hk(num_orders, d_off.p, d_base.p, ddist, dlen, droute, d_flag.p, nmax,
                        static_cast<uint32_t>(ctx->num_cus) * per_cu, st);
    }
    uint32_t ovf = 0;
    WR_HIP(hipMemcpyAsync(&ovf, d_flag.p, 4, hipMemcpyDeviceToHost, st));
    if (!dev) {
        WR_HIP(hipMemcpyAsync(length_out, dlen, static_cast<size_t>(num_orders) * 8, hipMemcpyDeviceToHost, st));
        if (total) WR_HIP(hipMemcpyAsync(route_out, droute, static_cast<size_t>(total) * 4, hipMemcpyDeviceToHost, st));
    }
    WR_HIP(hipStreamSynchronize(st));
    if (ovf) fail(WR_E_RANGE, "a partial route length reached 2^32-1 (lengths are accumulated in 32 bits)");
    WR_API_END
}

extern "C" wr_status wr_order_routes_clustered(wr_context *ctx, uint32_t num_orders, const uint32_t *pick_offsets,
                                               const uint32_t *dist, const int32_t *pick_xy, uint32_t m,
                                               uint64_t *length_out, uint32_t *route_out, uint32_t *clusters_out,
                                               uint32_t flags, void *stream) {
    WR_API_BEGIN
    if (!ctx) fail(WR_E_INVALID, "context is NULL");
    if (flags & ~static_cast<uint32_t>(WR_DEVICE_PTRS))
        fail(WR_E_INVALID, "unknown flags for wr_order_routes_clustered");
    if (m < 1 || m > route_clustered_max_clusters())
        fail(WR_E_INVALID, "m must be between 1 and " + std::to_string(route_clustered_max_clusters()));
    if (num_orders == 0) return WR_OK;
    const RouteBatch rb = route_batch(num_orders, pick_offsets, route_clustered_max_stops(), "clustered routes");
    const uint64_t cells = rb.cells;
    const uint32_t total = rb.total;
    if (!length_out) fail(WR_E_INVALID, "length_out is NULL");
    if (total && (!route_out || !pick_xy)) fail(WR_E_INVALID, "route_out or pick_xy is NULL");
    if (cells && !dist) fail(WR_E_INVALID, "dist is NULL");
    const bool dev = flags & WR_DEVICE_PTRS;
    if (!dev)
        for (uint64_t q = 0; q < 2ull * total; ++q)
            if (pick_xy[q] <= -65536 || pick_xy[q] >= 65536) fail(WR_E_RANGE, "pick positions must be below 2^16");
    WR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    join_caller_stream(ctx, dev, stream);
    DBuf<uint32_t> d_off, d_err, d_dist, d_route, d_m;
    DBuf<uint64_t> d_base, d_len;
    DBuf<int32_t> d_xy;
    upload(d_off, ctx, rb.off, st);
    upload(d_base, ctx, rb.mbase, st);
    d_err.alloc(ctx, 1);
    launch_fill_u32(d_err.p, 1, 0u, st);
    d_m.alloc(ctx, num_orders);
    const uint32_t *ddist = dist;
    const int32_t *dxy = pick_xy;
    uint64_t *dlen = length_out;
    uint32_t *droute = route_out;
    if (!dev) {
        d_dist.alloc(ctx, std::max<uint64_t>(cells, 1));
        if (cells) WR_HIP(hipMemcpyAsync(d_dist.p, dist, cells * 4, hipMemcpyHostToDevice, st));
        d_xy.alloc(ctx, std::max(2u * total, 2u));
        if (total) WR_HIP(hipMemcpyAsync(d_xy.p, pick_xy, 8ull * total, hipMemcpyHostToDevice, st));
        d_len.alloc(ctx, num_orders);
        d_route.alloc(ctx, std::max(total, 1u));
        ddist = d_dist.p;
        dxy = d_xy.p;
        dlen = d_len.p;
        droute = d_route.p;
    }
    launch_route_clustered(num_orders, d_off.p, d_base.p, ddist, dxy, m, dlen, droute, d_m.p, d_err.p,
                           static_cast<uint32_t>(ctx->num_cus), st);
    uint32_t err = 0;
    WR_HIP(hipMemcpyAsync(&err, d_err.p, 4, hipMemcpyDeviceToHost, st));
    std::vector<uint32_t> hm(num_orders);
    WR_HIP(hipMemcpyAsync(hm.data(), d_m.p, 4ull * num_orders, hipMemcpyDeviceToHost, st));
    if (!dev) {
        WR_HIP(hipMemcpyAsync(length_out, dlen, static_cast<size_t>(num_orders) * 8, hipMemcpyDeviceToHost, st));
        if (total) WR_HIP(hipMemcpyAsync(route_out, droute, static_cast<size_t>(total) * 4, hipMemcpyDeviceToHost, st));
    }
    WR_HIP(hipStreamSynchronize(st));
    if (err & 1u) fail(WR_E_RANGE, "a pick position is out of range or a cluster route length reached 2^32-1");
    if (err & 2u)
        fail(WR_E_UNSUPPORTED, "an order cannot be split into clusters of at most " +
                                   std::to_string(route_max_stops()) + " stops with at most " +
                                   std::to_string(route_clustered_max_clusters()) + " clusters");
    if (clusters_out) std::copy(hm.begin(), hm.end(), clusters_out);
    WR_API_END
}

// ------------------------------------------------------------------------
// wr_order_routes_static: wr_order_routes for callers that cannot allocate.
// Its work buffers (the orders' pick offsets and matrix bases, the overflow
// flag and, when enumerating, the per-order keys) live in one fixed device
// array, `scratch`, instead of allocations.  Host code never passes the
// array's name to a kernel: it takes the array's device address once per
// device with hipGetSymbolAddress and uses that address everywhere.
namespace {

constexpr uint32_t kStaticMaxOrders = WR_ROUTES_STATIC_MAX_ORDERS;
// [flag u32, padded to 256 B][off u32 x (max+1), padded][mbase u64 x max][key u64 x max]
constexpr size_t kScratchFlag = 0;
constexpr size_t kScratchOff = 256;
constexpr size_t kScratchBase = kScratchOff + ((4ull * (kStaticMaxOrders + 1) + 255) / 256) * 256;
constexpr size_t kScratchKey = kScratchBase + 8ull * kStaticMaxOrders;
constexpr size_t kScratchBytes = kScratchKey + 8ull * kStaticMaxOrders;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), taken once.
unsigned char *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) fail(WR_E_UNSUPPORTED, "device index beyond the static route buffers");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(WR_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    }
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" wr_status wr_order_routes_static(wr_context *ctx, uint32_t num_orders, const uint32_t *pick_offsets,
                                            const uint32_t *dist, uint64_t *length_out, uint32_t *route_out,
                                            uint32_t flags, void *stream) {
    WR_API_BEGIN
    if (!ctx) fail(WR_E_INVALID, "context is NULL");
    if (flags & ~static_cast<uint32_t>(WR_ROUTE_ENUMERATE))
        fail(WR_E_INVALID, "unknown flags for wr_order_routes_static");
    if (num_orders == 0) return WR_OK;
    if (num_orders > kStaticMaxOrders)
        fail(WR_E_RANGE, "wr_order_routes_static serves at most " + std::to_string(kStaticMaxOrders) +
                             " orders per call (asked for " + std::to_string(num_orders) + ")");
    const bool enumerate = flags & WR_ROUTE_ENUMERATE;
    const RouteBatch rb = route_batch(num_orders, pick_offsets,
                                      enumerate ? route_enumerate_max_stops() : route_max_stops(),
                                      enumerate ? "enumerated routes" : "exact routes");
    if (!length_out) fail(WR_E_INVALID, "length_out is NULL");
    if (rb.total && !route_out) fail(WR_E_INVALID, "route_out is NULL");
    if (rb.cells && !dist) fail(WR_E_INVALID, "dist is NULL");
    WR_HIP(hipSetDevice(ctx->device));
    unsigned char *base = scratch_on(ctx->device);
    uint32_t *d_flag = reinterpret_cast<uint32_t *>(base + kScratchFlag);
    uint32_t *d_off = reinterpret_cast<uint32_t *>(base + kScratchOff);
    uint64_t *d_base = reinterpret_cast<uint64_t *>(base + kScratchBase);
    unsigned long long *d_key = reinterpret_cast<unsigned long long *>(base + kScratchKey);
    // everything runs on the caller's stream, in order after its earlier work
    hipStream_t st = static_cast<hipStream_t>(stream);
    WR_HIP(hipMemcpyAsync(d_off, rb.off.data(), 4ull * (num_orders + 1), hipMemcpyHostToDevice, st));
    WR_HIP(hipMemcpyAsync(d_base, rb.mbase.data(), 8ull * num_orders, hipMemcpyHostToDevice, st));
    launch_fill_u32(d_flag, 1, 0u, st);
    if (enumerate) {
        launch_fill_u32(reinterpret_cast<uint32_t *>(d_key), 2ull * num_orders, 0xFFFFFFFFu, st);
        launch_route_perm(num_orders, d_off, d_base, dist, d_key, length_out, route_out, d_flag, rb.nmax, st);
    } else {
        const uint32_t lds = route_lds_bytes(std::max(rb.nmax, 1u));
        const uint32_t per_cu = std::max(1u, std::min(8u, (160u * 1024u) / lds));
        launch_route_hk(num_orders, d_off, d_base, dist, length_out, route_out, d_flag, rb.nmax,
                        static_cast<uint32_t>(ctx->num_cus) * per_cu, st);
    }
    // the host copies above read rb's vectors, and the flag decides the
    // status: wait for the stream before returning
    uint32_t ovf = 0;
    WR_HIP(hipMemcpyAsync(&ovf, d_flag, 4, hipMemcpyDeviceToHost, st));
    WR_HIP(hipStreamSynchronize(st));
    if (ovf) fail(WR_E_RANGE, "a partial route length reached 2^32-1 (lengths are accumulated in 32 bits)");
    WR_API_END
}
