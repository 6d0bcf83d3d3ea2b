// K-means over at most 64 integer points held one per lane of a wave.
//
// The clustering step of the Route Optimization section (picks of an order)
// and of the restocking rule (purchase orders of a picking order) both use
// this reading of K-means: the first centre is point 0, each further centre
// is the point farthest from the centres so far (ties to the smaller index),
// then Lloyd steps -- every point to its nearest centre, ties to the smaller
// cluster, each non-empty cluster's centre to the mean of its points -- until
// no point changes cluster, at most 100 steps.  Centres are kept as (sum x,
// sum y, count) and distances are compared exactly in 64-bit integers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wr {

constexpr int KM_MAX_STEPS = 100;

// value of v held by lane src of the wave (two 32-bit shuffles)
__device__ __forceinline__ int64_t km_shfl64(int64_t v, uint32_t src) {
    const uint32_t lo = __shfl(static_cast<uint32_t>(static_cast<uint64_t>(v)), static_cast<int>(src), 64);
    const uint32_t hi = __shfl(static_cast<uint32_t>(static_cast<uint64_t>(v) >> 32), static_cast<int>(src), 64);
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// sign of |p - Sa/ca|^2 - |p - Sb/cb|^2, with both sides multiplied by
// (ca cb)^2 so that it stays in integers.  Exact while
// 2 (count * coordinate bound)^2 * count^2 < 2^63.
__device__ __forceinline__ int km_cmp(int64_t px, int64_t py, int64_t sxa, int64_t sya, int64_t ca, int64_t sxb,
                                      int64_t syb, int64_t cb) {
    const int64_t dxa = ca * px - sxa, dya = ca * py - sya;
    const int64_t dxb = cb * px - sxb, dyb = cb * py - syb;
    const int64_t a = (dxa * dxa + dya * dya) * (cb * cb);
    const int64_t b = (dxb * dxb + dyb * dyb) * (ca * ca);
    return a < b ? -1 : (a > b ? 1 : 0);
}

// Every lane of the wave calls this with its point (px, py); lanes with
// on == false (lane >= n) take no part.  xy: the n points as int32 pairs in
// LDS; cen: LDS scratch of 3 m int64; asg: LDS [n], left holding every
// point's cluster.  Returns this lane's cluster (0xFFFFFFFF when !on).
// Clusters are numbered below min(m, n).
__device__ inline uint32_t wave_kmeans(bool on, int64_t px, int64_t py, uint32_t n, uint32_t m, const int32_t *xy,
                                       int64_t *cen, uint32_t *asg) {
    const uint32_t lane = threadIdx.x & 63u;
    // farthest-point initial centres
    int64_t dmin = INT64_MAX;
    uint32_t nc = 0, c0 = 0;
    for (;;) {
        const int64_t cx = xy[2 * c0], cy = xy[2 * c0 + 1];
        if (lane == 0) {
            cen[3 * nc] = cx;
            cen[3 * nc + 1] = cy;
            cen[3 * nc + 2] = 1;
        }
        ++nc;
        if (nc >= m || nc >= n) break;
        const int64_t dx = px - cx, dy = py - cy;
        const int64_t d = dx * dx + dy * dy;
        if (on && d < dmin) dmin = d;
        int64_t best = on ? dmin : -1;
        uint32_t bi = lane;
        for (uint32_t sh = 1; sh < 64; sh <<= 1) {
            const int64_t ob = km_shfl64(best, lane ^ sh);
            const uint32_t oi = __shfl(bi, static_cast<int>(lane ^ sh), 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        c0 = bi;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t a = 0xFFFFFFFFu;
    for (int it = 0; it < KM_MAX_STEPS; ++it) {
        uint32_t b = 0;
        for (uint32_t c = 1; c < nc; ++c)
            if (km_cmp(px, py, cen[3 * c], cen[3 * c + 1], cen[3 * c + 2], cen[3 * b], cen[3 * b + 1],
                       cen[3 * b + 2]) < 0)
                b = c;
        const bool ch = on && a != b;
        if (on) a = b;
        if (__builtin_amdgcn_ballot_w64(ch) == 0) break;
        if (on) asg[lane] = a;
        __builtin_amdgcn_wave_barrier();
        // lane c < nc sums its cluster's points; empty clusters keep their centre
        if (lane < nc) {
            int64_t sx = 0, sy = 0, cn = 0;
            for (uint32_t i = 0; i < n; ++i)
                if (asg[i] == lane) {
                    sx += xy[2 * i];
                    sy += xy[2 * i + 1];
                    ++cn;
                }
            if (cn) {
                cen[3 * lane] = sx;
                cen[3 * lane + 1] = sy;
                cen[3 * lane + 2] = cn;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (on) asg[lane] = a;
    __builtin_amdgcn_wave_barrier();
    return a;
}

}  // namespace wr
