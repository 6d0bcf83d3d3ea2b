// CPU executor for the library's HIP kernels -- TEST INFRASTRUCTURE ONLY.
//
// Put this directory first on the include path and compile the unchanged
// library sources as plain C++ (g++ -x c++, with AddressSanitizer): every
// kernel launch then runs on the CPU, one OS thread per lane, with wave
// collectives (ballot, readfirstlane, wave barrier) and __syncthreads
// emulated by barriers, and every device allocation is an ordinary heap
// block that ASan bounds-checks.  It exists to find out-of-bounds accesses
// and logic errors of the kernels and the host runtime without a GPU; it is
// never loaded by the product package.
#pragma once

#include <algorithm>
#include <atomic>
#include <barrier>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <type_traits>
#include <vector>

#define __global__
#define __device__
#define __align__(n) alignas(n)
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

struct dim3 {
    unsigned x, y, z;
    constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint2 {
    unsigned x, y;
};
struct uint4 {
    unsigned x, y, z, w;
};
inline uint2 make_uint2(unsigned a, unsigned b) { return {a, b}; }
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return {a, b, c, d}; }

namespace simt {

struct Wave {
    std::unique_ptr<std::barrier<>> bar;
    uint64_t vals[64];
    bool alive[64];
    unsigned n = 0;
};

struct Block {
    std::unique_ptr<std::barrier<>> bar;
    std::vector<Wave> waves;
};

struct Lane {
    dim3 tid, bid, bdim, gdim;
    Block *blk = nullptr;
    unsigned wave = 0, lane = 0;
    volatile int line = 0;    // source line of the last collective entered
    volatile int waiting = 0; // 1 = in a wave collective, 2 = in __syncthreads
};
extern std::atomic<unsigned long> progress;

extern thread_local Lane *cur;

inline Wave &wave() { return cur->blk->waves[cur->wave]; }

inline uint64_t ballot(bool p, int line = 0) {
    cur->line = line;
    Wave &w = wave();
    w.vals[cur->lane] = p ? 1u : 0u;
    w.bar->arrive_and_wait();
    uint64_t m = 0;
    for (unsigned l = 0; l < w.n; ++l)
        if (w.alive[l] && w.vals[l]) m |= 1ull << l;
    w.bar->arrive_and_wait();
    progress++;
    return m;
}

inline uint32_t readfirstlane(uint32_t x, int line = 0) {
    cur->line = line;
    Wave &w = wave();
    w.vals[cur->lane] = x;
    w.bar->arrive_and_wait();
    uint32_t r = 0;
    for (unsigned l = 0; l < w.n; ++l)
        if (w.alive[l]) {
            r = static_cast<uint32_t>(w.vals[l]);
            break;
        }
    w.bar->arrive_and_wait();
    progress++;
    return r;
}

inline void wave_barrier(int line = 0) {
    cur->line = line;
    cur->waiting = 1;
    wave().bar->arrive_and_wait();
    cur->waiting = 0;
    progress++;
}

// value of `x` held by lane `src` (lanes outside the wave read their own)
inline uint32_t shfl(uint32_t x, int src, int line = 0) {
    cur->line = line;
    Wave &w = wave();
    w.vals[cur->lane] = x;
    w.bar->arrive_and_wait();
    const unsigned s = static_cast<unsigned>(src) & 63u;
    const uint32_t r = s < w.n ? static_cast<uint32_t>(w.vals[s]) : x;
    w.bar->arrive_and_wait();
    progress++;
    return r;
}
// DPP move within a row of 16 lanes: quad permutations, row and half-row
// mirrors (the patterns the library uses; all lanes active)
inline uint32_t update_dpp(uint32_t, uint32_t src, int ctrl) {
    const unsigned l = cur->lane;
    unsigned s;
    if (ctrl < 0x100) s = (l & ~3u) | ((static_cast<unsigned>(ctrl) >> (2 * (l & 3u))) & 3u);
    else if (ctrl == 0x140) s = (l & ~15u) | (15u - (l & 15u));
    else if (ctrl == 0x141) s = (l & ~7u) | (7u - (l & 7u));
    else std::abort();
    return shfl(src, static_cast<int>(s));
}
inline uint32_t shfl_xor(uint32_t x, unsigned m) { return shfl(x, static_cast<int>(cur->lane ^ m)); }
inline uint32_t shfl_up(uint32_t x, unsigned d) {
    const unsigned l = cur->lane;
    const uint32_t r = shfl(x, l >= d ? static_cast<int>(l - d) : static_cast<int>(l));
    return r;
}
inline void syncthreads(int line = 0) {
    cur->line = line;
    cur->waiting = 2;
    cur->blk->bar->arrive_and_wait();
    cur->waiting = 0;
    progress++;
}

inline uint32_t mbcnt_lo(uint32_t m, uint32_t a) {
    const unsigned l = cur->lane;
    const uint32_t mask = l >= 32 ? 0xFFFFFFFFu : ((1u << l) - 1u);
    return a + static_cast<uint32_t>(__builtin_popcount(m & mask));
}
inline uint32_t mbcnt_hi(uint32_t m, uint32_t a) {
    const unsigned l = cur->lane;
    const uint32_t mask = l < 32 ? 0u : ((1u << (l - 32)) - 1u);
    return a + static_cast<uint32_t>(__builtin_popcount(m & mask));
}

template <class T>
inline T add_sat(T a, T b) {
    T r = a + b;
    return r < a ? static_cast<T>(~T(0)) : r;
}

void run_grid(dim3 g, dim3 b, const std::function<void()> &body);

struct Job {
    std::function<void()> fn;
};
bool capturing(void *stream);
void record(void *stream, std::function<void()> fn);

}  // namespace simt

#define threadIdx (::simt::cur->tid)
#define blockIdx (::simt::cur->bid)
#define blockDim (::simt::cur->bdim)
#define gridDim (::simt::cur->gdim)
#define __syncthreads() ::simt::syncthreads(__LINE__)
#define __shfl(x, src, w) ::simt::shfl((x), (src), __LINE__)
#define __shfl_up(x, d, w) ::simt::shfl_up((x), (d))
#define __shfl_xor(x, m, w) ::simt::shfl_xor((x), static_cast<unsigned>(m))
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) ::simt::update_dpp((old), (src), (ctrl))
#define __builtin_amdgcn_ballot_w64(p) ::simt::ballot((p), __LINE__)
#define __builtin_amdgcn_readfirstlane(x) ::simt::readfirstlane((x), __LINE__)
#define __builtin_amdgcn_readlane(x, k) ::simt::shfl((x), static_cast<int>(k), __LINE__)
#define __builtin_amdgcn_wave_barrier() ::simt::wave_barrier(__LINE__)
#define __builtin_amdgcn_mbcnt_lo(m, a) ::simt::mbcnt_lo(m, a)
#define __builtin_amdgcn_mbcnt_hi(m, a) ::simt::mbcnt_hi(m, a)
#define __builtin_elementwise_add_sat(a, b) ::simt::add_sat(a, b)
#define __HIP_MEMORY_SCOPE_WAVEFRONT 1
#define __HIP_MEMORY_SCOPE_WORKGROUP 2
#define __HIP_MEMORY_SCOPE_AGENT 3
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)

template <class T, class U>
inline T atomicAdd(T *p, U v) { return __atomic_fetch_add(p, static_cast<T>(v), __ATOMIC_SEQ_CST); }
template <class T, class U>
inline T atomicOr(T *p, U v) { return __atomic_fetch_or(p, static_cast<T>(v), __ATOMIC_SEQ_CST); }
template <class T, class U>
inline T atomicAnd(T *p, U v) { return __atomic_fetch_and(p, static_cast<T>(v), __ATOMIC_SEQ_CST); }
template <class T, class U, class V>
inline T atomicCAS(T *p, U cmp, V val) {
    T old = static_cast<T>(cmp);
    __atomic_compare_exchange_n(p, &old, static_cast<T>(val), false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
    return old;
}
template <class T, class U>
inline T atomicMin(T *p, U vv) {
    const T v = static_cast<T>(vv);
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v < old && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return old;
}
template <class T, class U>
inline T atomicMax(T *p, U vv) {
    const T v = static_cast<T>(vv);
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v > old && !__atomic_compare_exchange_n(p, &old, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return old;
}
inline uint32_t min(uint32_t a, uint32_t b) { return a < b ? a : b; }
inline uint32_t max(uint32_t a, uint32_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------- runtime API
typedef int hipError_t;
enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNoDevice = 100,
    hipErrorLaunchFailure = 719
};
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
typedef struct ihipGraph *hipGraph_t;
typedef struct ihipGraphExec *hipGraphExec_t;
typedef struct ihipGraphNode *hipGraphNode_t;
struct hipDeviceProp_t {
    char name[256];
    int multiProcessorCount;
    size_t totalGlobalMem;
};
enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
};
enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2
};
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0
#define hipEventRecordExternal 0x01

hipError_t hipGetDeviceCount(int *n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int *d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int d);
hipError_t hipMemGetInfo(size_t *freeb, size_t *total);
hipError_t hipMalloc(void **p, size_t n);
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t n, unsigned flags);
hipError_t hipHostFree(void *p);
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned f);
hipError_t hipStreamCreate(hipStream_t *s);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned f);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned f);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventRecordWithFlags(hipEvent_t e, hipStream_t s, unsigned flags);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, hipGraphNode_t *n, char *log, size_t sz);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
// device variables are host objects here: a symbol's address is its own
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
    *p = const_cast<void *>(sym);
    return hipSuccess;
}

namespace simt {
void trace(const char *name, dim3 g, dim3 b, double ms);
double now_ms();
// dynamic LDS of the running launch (blocks run one after another)
void set_dynamic_lds(size_t bytes);
void *dynamic_lds();
template <class... P, class... A>
void launch(const char *name, void (*k)(P...), dim3 g, dim3 b, size_t sh, hipStream_t st, A &&...a) {
    std::tuple<std::decay_t<P>...> args(static_cast<std::decay_t<P>>(a)...);
    std::function<void()> job = [name, k, g, b, sh, args]() {
        const double t0 = now_ms();
        set_dynamic_lds(sh);
        run_grid(g, b, [&]() { std::apply(k, args); });
        trace(name, g, b, now_ms() - t0);
    };
    if (capturing(st))
        record(st, std::move(job));
    else
        job();
}
}  // namespace simt

#define HIP_KERNEL_NAME(...) __VA_ARGS__
#define hipLaunchKernelGGL(k, g, b, sh, st, ...) \
    ::simt::launch(#k, k, ::dim3(g), ::dim3(b), static_cast<size_t>(sh), (st), ##__VA_ARGS__)
#define HIP_DYNAMIC_SHARED(type, var) type *var = static_cast<type *>(::simt::dynamic_lds());
