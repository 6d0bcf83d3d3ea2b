// CPU executor runtime (see hip/hip_runtime.h) -- TEST INFRASTRUCTURE ONLY.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <map>
#include <mutex>

namespace simt {

thread_local Lane *cur = nullptr;
std::atomic<unsigned long> progress{0};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

void trace(const char *name, dim3 g, dim3 b, double ms) {
    static const bool on = std::getenv("SIMT_TRACE") != nullptr;
    if (on) std::fprintf(stderr, "[simt] %s grid=(%u,%u,%u) block=%u %.1f ms\n", name, g.x, g.y, g.z, b.x * b.y * b.z, ms);
}

namespace {
std::vector<uint64_t> g_dyn_lds;
}
void set_dynamic_lds(size_t bytes) {
    g_dyn_lds.assign((bytes + 7) / 8, 0xDEADBEEFDEADBEEFull);
}
void *dynamic_lds() { return g_dyn_lds.empty() ? nullptr : g_dyn_lds.data(); }

void run_grid(dim3 g, dim3 b, const std::function<void()> &body) {
    const unsigned nt = b.x * b.y * b.z;
    for (unsigned bz = 0; bz < g.z; ++bz)
        for (unsigned by = 0; by < g.y; ++by)
            for (unsigned bx = 0; bx < g.x; ++bx) {
                Block blk;
                blk.bar = std::make_unique<std::barrier<>>(nt);
                const unsigned nw = (nt + 63) / 64;
                blk.waves.resize(nw);
                for (unsigned w = 0; w < nw; ++w) {
                    const unsigned n = std::min(64u, nt - 64 * w);
                    blk.waves[w].n = n;
                    blk.waves[w].bar = std::make_unique<std::barrier<>>(n);
                    for (unsigned l = 0; l < 64; ++l) blk.waves[w].alive[l] = l < n;
                }
                std::vector<Lane *> lanes(nt, nullptr);
                std::atomic<bool> done{false};
                std::thread dog([&]() {
                    unsigned long last = progress.load();
                    int idle = 0;
                    while (!done.load()) {
                        std::this_thread::sleep_for(std::chrono::milliseconds(200));
                        const unsigned long p = progress.load();
                        if (p != last) { last = p; idle = 0; continue; }
                        if (++idle < 25) continue;
                        std::fprintf(stderr, "[simt] no barrier progress for 5 s in block (%u,%u,%u)\n", bx, by, bz);
                        std::map<std::pair<int, int>, int> hist;
                        for (unsigned t = 0; t < nt; ++t)
                            if (lanes[t]) hist[{lanes[t]->line, lanes[t]->waiting}]++;
                            else hist[{-1, -1}]++;
                        for (auto &kv : hist)
                            std::fprintf(stderr, "[simt]   line %d waiting %d : %d lanes\n", kv.first.first, kv.first.second, kv.second);
                        std::abort();
                    }
                });
                std::vector<std::thread> th;
                th.reserve(nt);
                for (unsigned t = 0; t < nt; ++t) {
                    th.emplace_back([&, t]() {
                        Lane ln;
                        ln.tid = dim3(t % b.x, (t / b.x) % b.y, t / (b.x * b.y));
                        ln.bid = dim3(bx, by, bz);
                        ln.bdim = b;
                        ln.gdim = g;
                        ln.blk = &blk;
                        ln.wave = t / 64;
                        ln.lane = t % 64;
                        cur = &ln;
                        lanes[t] = &ln;
                        body();
                        Wave &w = blk.waves[ln.wave];
                        w.alive[ln.lane] = false;
                        w.bar->arrive_and_drop();
                        blk.bar->arrive_and_drop();
                        progress++;
                        lanes[t] = nullptr;
                        cur = nullptr;
                    });
                }
                for (auto &x : th) x.join();
                done = true;
                dog.join();
            }
}

static std::mutex g_mu;
static std::map<void *, std::vector<std::function<void()>> *> g_capture;

bool capturing(void *s) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_capture.count(s) != 0;
}
void record(void *s, std::function<void()> fn) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_capture[s]->push_back(std::move(fn));
}

}  // namespace simt

struct ihipStream_t { int dummy; };
struct ihipEvent_t { int dummy; };
struct ihipGraph { std::vector<std::function<void()>> jobs; };
struct ihipGraphExec { std::vector<std::function<void()>> jobs; };

hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
    std::memset(p, 0, sizeof(*p));
    std::strcpy(p->name, "cpu-simt");
    p->multiProcessorCount = 2;
    p->totalGlobalMem = 8ull << 30;
    return hipSuccess;
}
hipError_t hipMemGetInfo(size_t *f, size_t *t) { *f = 4ull << 30; *t = 8ull << 30; return hipSuccess; }
hipError_t hipMalloc(void **p, size_t n) { *p = std::malloc(n ? n : 1); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { if (n) std::memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st) {
    if (simt::capturing(st)) {
        simt::record(st, [d, s, n]() { if (n) std::memcpy(d, s, n); });
        return hipSuccess;
    }
    return hipMemcpy(d, s, n, k);
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { std::memset(d, v, n); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new ihipStream_t(); return hipSuccess; }
hipError_t hipStreamCreate(hipStream_t *s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) { *e = new ihipEvent_t(); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventRecordWithFlags(hipEvent_t, hipStream_t, unsigned) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "success" : "simulated error"; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    std::lock_guard<std::mutex> lk(simt::g_mu);
    simt::g_capture[s] = new std::vector<std::function<void()>>();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    std::lock_guard<std::mutex> lk(simt::g_mu);
    auto it = simt::g_capture.find(s);
    if (it == simt::g_capture.end()) { *g = nullptr; return hipErrorInvalidValue; }
    *g = new ihipGraph();
    (*g)->jobs = std::move(*it->second);
    delete it->second;
    simt::g_capture.erase(it);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    *e = new ihipGraphExec();
    (*e)->jobs = g->jobs;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
    for (auto &j : e->jobs) j();
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
