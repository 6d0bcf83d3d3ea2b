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

#include "wave_ops.hpp"

namespace wr {

constexpr int KM_MAX_STEPS = 100;

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
// on == false (lane >= n) take no part.  Coordinates must lie in
// (-2^25, 2^25) and counts times coordinates in 32 bits.  xy: the n points
// as int32 pairs in LDS; cen: LDS scratch of 3 m int64; asg: LDS [n], left
// holding every point's cluster.  Returns this lane's cluster (0xFFFFFFFF
// when !on).  Clusters are numbered below min(m, n).
__device__ inline uint32_t wave_kmeans(bool on, int64_t px, int64_t py, uint32_t n, uint32_t m, const int32_t *xy,
                                       int64_t *cen, uint32_t *asg) {
    const uint32_t lane = threadIdx.x & 63u;
    const int32_t px32 = static_cast<int32_t>(px), py32 = static_cast<int32_t>(py);
    // farthest-point initial centres: the key (d + 1) << 6 | (63 - lane)
    // orders points by their distance to the nearest centre so far, ties to
    // the smaller index, and puts every point above the lanes past n
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
        const uint64_t key = on ? ((static_cast<uint64_t>(dmin) + 1) << 6) | (63u - lane) : 0;
        c0 = 63u - static_cast<uint32_t>(wave_max_u64(key) & 63u);
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
        // lane c < nc sums its cluster's points (broadcast from their lanes);
        // empty clusters keep their centre
        int32_t sx = 0, sy = 0, cn = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t ai = __builtin_amdgcn_readlane(a, i);
            const int32_t xi = __builtin_amdgcn_readlane(px32, i), yi = __builtin_amdgcn_readlane(py32, i);
            if (ai == lane) {
                sx += xi;
                sy += yi;
                ++cn;
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < nc && cn) {
            cen[3 * lane] = sx;
            cen[3 * lane + 1] = sy;
            cen[3 * lane + 2] = cn;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (on) asg[lane] = a;
    __builtin_amdgcn_wave_barrier();
    return a;
}

}  // namespace wr
