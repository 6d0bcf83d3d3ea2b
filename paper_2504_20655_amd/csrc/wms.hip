// wr_wms_run: the warehouse reorganisation loop -- the random dynamical
// system x_n = f(o_n, x_{n-1}) of the Mathematical model section, one
// application of f per picking order: cluster the order's purchase orders by
// where their articles are stored, fill the order (the map w), and restock
// every node whose last parcel a pick would take at the empty node nearest
// its cluster's centre when that node is strictly nearer (the restocking
// rule of the Clustering section; order processing, stock update and
// check-and-move of the WMS loop appendix).
//
// One wave per run, every iteration in the same launch:
//   * the state stays in HBM (A, M, and pos[article] = node in a scratch
//     array); per iteration only the order's slots are gathered into LDS;
//   * the empty nodes are one bitmask of empty shelves per rack, kept in LDS
//     for the whole run, so a nearest-empty query scans racks in a window
//     around the centre that grows until nothing outside it can be as near;
//   * each cluster's nearest empty node is cached: a query is a compare,
//     and a move updates the caches (the vacated node can only lower them,
//     the taken node invalidates the caches that held it);
//   * the picks run in order on one wave with the slot values broadcast from
//     registers; an article picked twice in one order keeps its live state in
//     an LDS hash cell.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kmeans_wave.hpp"
#include "wr_internal.hpp"

namespace wr {
namespace {

constexpr uint32_t WMS_KMAX = 10;          // clusters
constexpr uint32_t WMS_POMAX = 64;         // purchase orders: one K-means point per lane
constexpr uint32_t WMS_SMAX = 1024;        // slots (purchase orders x articles) per order
constexpr uint32_t WMS_MASK_BYTES = 65536; // LDS for the rack masks
constexpr uint64_t NOKEY = ~0ull;
constexpr uint32_t DUP = 0x80000000u;
constexpr uint32_t WMS_ERR_STATE = 1u, WMS_ERR_ORDER = 2u;

struct WmsArgs {
    uint32_t nx, ny, nz, n_articles, mmax, po, per, k, iters, S, H;
    uint32_t *A, *M;                         // [runs][V]
    const uint32_t *orders, *qty;            // [runs][iters][S]
    uint32_t *pos;                           // [runs][N + 1] scratch
    double *sil, *area;                      // [runs][iters]
    uint32_t *moves;                         // [runs][iters]
    uint32_t *err;
};

// packed rack position of a node: i | j << 11 | k << 22
__device__ __forceinline__ uint32_t pack_ijk(uint32_t i, uint32_t j, uint32_t k) { return i | (j << 11) | (k << 22); }
__device__ __forceinline__ uint32_t ijk_i(uint32_t p) { return p & 2047u; }
__device__ __forceinline__ uint32_t ijk_j(uint32_t p) { return (p >> 11) & 2047u; }
__device__ __forceinline__ uint32_t ijk_k(uint32_t p) { return p >> 22; }

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
    for (uint32_t sh = 1; sh < 64; sh <<= 1) {
        const uint32_t lo = __shfl_xor(static_cast<uint32_t>(x), static_cast<int>(sh), 64);
        const uint32_t hi = __shfl_xor(static_cast<uint32_t>(x >> 32), static_cast<int>(sh), 64);
        const uint64_t o = (static_cast<uint64_t>(hi) << 32) | lo;
        x = o < x ? o : x;
    }
    return x;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// squared distance of rack (i, j) to the centre S / scale, times scale^2
__device__ __forceinline__ uint64_t centre_d2(uint32_t i, uint32_t j, int64_t sx, int64_t sy, int64_t scale) {
    const int64_t dx = scale * static_cast<int64_t>(i) - sx, dy = scale * static_cast<int64_t>(j) - sy;
    return static_cast<uint64_t>(dx * dx + dy * dy);
}

// Empty shelves of rack r: MPW masks of 32 / MPW bits per 4-byte LDS word.
template <uint32_t MPW>
__device__ __forceinline__ uint32_t rack_mask(const uint32_t *mword, uint32_t r) {
    if constexpr (MPW == 1) return mword[r];
    else return (mword[r >> 1] >> ((r & 1u) * 16u)) & 0xFFFFu;
}
template <uint32_t MPW>
__device__ __forceinline__ uint32_t rack_bit(uint32_t r, uint32_t k) {
    return (1u << k) << ((32u / MPW) * (r % MPW));
}

// The empty node nearest the centre (sx, sy) / scale as the key
// d2 << 24 | node (ties to the smaller node id: the lowest empty shelf of the
// rack, then the rack order), NOKEY when no node is empty.  Racks are scanned
// in a window around the centre's rack, 8 x 8 racks per step of the wave;
// the window doubles until the best key found is nearer than any rack
// outside it can be.
template <uint32_t MPW>
__device__ uint64_t nearest_empty(const uint32_t *mword, uint32_t nx, uint32_t ny, int64_t sx, int64_t sy,
                                  int64_t scale) {
    const uint32_t lane = threadIdx.x & 63u;
    const int32_t ci = static_cast<int32_t>(std::min<int64_t>(sx / scale, static_cast<int64_t>(nx) - 1));
    const int32_t cj = static_cast<int32_t>(std::min<int64_t>(sy / scale, static_cast<int64_t>(ny) - 1));
    int32_t R = 3;
    for (;;) {
        const int32_t i0 = std::max(ci - R, 0), i1 = std::min(ci + R, static_cast<int32_t>(nx) - 1);
        const int32_t j0 = std::max(cj - R, 0), j1 = std::min(cj + R, static_cast<int32_t>(ny) - 1);
        uint64_t best = NOKEY;
        for (int32_t jb = j0; jb <= j1; jb += 8)
            for (int32_t ib = i0; ib <= i1; ib += 8) {
                const int32_t i = ib + static_cast<int32_t>(lane & 7u), j = jb + static_cast<int32_t>(lane >> 3);
                if (i <= i1 && j <= j1) {
                    const uint32_t mk = rack_mask<MPW>(mword, static_cast<uint32_t>(j) * nx + static_cast<uint32_t>(i));
                    if (mk) {
                        const uint32_t k = __builtin_ctz(mk);
                        const uint32_t node = (k * ny + static_cast<uint32_t>(j)) * nx + static_cast<uint32_t>(i);
                        const uint64_t key = (centre_d2(i, j, sx, sy, scale) << 24) | node;
                        best = key < best ? key : best;
                    }
                }
            }
        best = uniform64(wave_min_u64(best));
        // nearest any rack outside the window can be (the centre lies in
        // the window's column and row ranges)
        uint64_t lb = NOKEY;
        if (i0 > 0) {
            const int64_t d = sx - scale * (i0 - 1);
            lb = std::min(lb, static_cast<uint64_t>(d * d));
        }
        if (i1 < static_cast<int32_t>(nx) - 1) {
            const int64_t d = scale * (i1 + 1) - sx;
            lb = std::min(lb, static_cast<uint64_t>(d * d));
        }
        if (j0 > 0) {
            const int64_t d = sy - scale * (j0 - 1);
            lb = std::min(lb, static_cast<uint64_t>(d * d));
        }
        if (j1 < static_cast<int32_t>(ny) - 1) {
            const int64_t d = scale * (j1 + 1) - sy;
            lb = std::min(lb, static_cast<uint64_t>(d * d));
        }
        if (lb == NOKEY || (best != NOKEY && (best >> 24) < lb)) return best;
        R = 2 * R + 1;
    }
}

template <uint32_t MPW>
__global__ __launch_bounds__(64) void k_wms(WmsArgs P) {
    HIP_DYNAMIC_SHARED(uint32_t, lds)
    const uint32_t lane = threadIdx.x;
    const uint32_t run = blockIdx.x;
    const uint32_t nx = P.nx, ny = P.ny, nz = P.nz, racks = nx * ny, V = racks * nz, N = P.n_articles;
    const uint32_t S = P.S, H = P.H, po = P.po, per = P.per;
    const uint32_t kc = std::min(P.k, po);   // clusters K-means can fill
    // ---- LDS: 8-byte arrays first
    int64_t *cen = reinterpret_cast<int64_t *>(lds);   // [3 KMAX] K-means scratch
    int64_t *cS = cen + 3 * WMS_KMAX;                   // [3 KMAX] sum x, sum y, count per cluster
    uint64_t *best = reinterpret_cast<uint64_t *>(cS + 3 * WMS_KMAX);   // [KMAX] nearest empty key
    double *sSil = reinterpret_cast<double *>(best + WMS_KMAX);          // [POMAX]
    uint32_t *sArt = reinterpret_cast<uint32_t *>(sSil + WMS_POMAX);     // [S]
    uint32_t *sQty = sArt + S, *sIJK = sQty + S, *sM = sIJK + S, *sCell = sM + S;
    uint32_t *hKey = sCell + S, *hCnt = hKey + H, *hIJK = hCnt + H, *hM = hIJK + H;
    uint32_t *sMov = hM + H;                     // [3 S] moves: from node, to node, article
    int32_t *xy = reinterpret_cast<int32_t *>(sMov + 3 * S);   // [2 POMAX]
    uint32_t *asg = reinterpret_cast<uint32_t *>(xy + 2 * WMS_POMAX);   // [POMAX]
    uint32_t *mword = asg + WMS_POMAX;           // rack masks, MPW per 4-byte word
    const uint32_t mwords = (racks + MPW - 1) / MPW;

    uint32_t *Ar = P.A + static_cast<size_t>(run) * V;
    uint32_t *Mr = P.M + static_cast<size_t>(run) * V;
    uint32_t *pos = P.pos + static_cast<size_t>(run) * (N + 1);

    // ---- set-up: pos[article] = node, the racks' empty shelves
    for (uint32_t w = lane; w < mwords; w += 64) mword[w] = 0;
    for (uint32_t a = lane; a <= N; a += 64) pos[a] = NONE;
    __syncthreads();
    bool bad = false;
    for (uint32_t k = 0; k < nz; ++k)
        for (uint32_t r = lane; r < racks; r += 64) {
            const uint32_t v = k * racks + r, a = Ar[v];
            if (a == 0)
                atomicOr(&mword[r / MPW], rack_bit<MPW>(r, k));
            else if (a > N)
                bad = true;
            else
                pos[a] = v;
        }
    __syncthreads();
    for (uint32_t v = lane; v < V; v += 64) {
        const uint32_t a = Ar[v];
        if (a != 0 && a <= N && pos[a] != v) bad = true;   // an article at two nodes
    }
    if (__builtin_amdgcn_ballot_w64(bad)) {
        if (lane == 0) atomicOr(P.err, WMS_ERR_STATE);
        return;
    }

    for (uint32_t it = 0; it < P.iters; ++it) {
        const size_t ob = (static_cast<size_t>(run) * P.iters + it) * S;
        for (uint32_t h = lane; h < H; h += 64) {
            hKey[h] = 0;
            hCnt[h] = 0;
        }
        __syncthreads();
        // ---- gather the order's slots: article, parcels, node, balance
        for (uint32_t s = lane; s < S; s += 64) {
            const uint32_t a = P.orders[ob + s], q = P.qty[ob + s];
            uint32_t v = (a >= 1 && a <= N) ? pos[a] : NONE;
            if (v == NONE || q > P.mmax) {
                bad = true;
                v = 0;
            }
            const uint32_t m = Mr[v];
            const uint32_t i = v % nx, t = v / nx;
            sArt[s] = a;
            sQty[s] = q;
            sIJK[s] = pack_ijk(i, t % ny, t / ny);
            sM[s] = m;
            uint32_t h = (a * 2654435761u) & (H - 1);
            for (;;) {
                const uint32_t old = atomicCAS(&hKey[h], 0u, a);
                if (old == 0u || old == a) break;
                h = (h + 1) & (H - 1);
            }
            atomicAdd(&hCnt[h], 1u);
            sCell[s] = h;
        }
        if (__builtin_amdgcn_ballot_w64(bad)) {
            if (lane == 0) atomicOr(P.err, WMS_ERR_ORDER);
            return;
        }
        __syncthreads();
        // an article picked more than once in this order: its live state in the cell
        for (uint32_t s = lane; s < S; s += 64) {
            const uint32_t h = sCell[s];
            if (hCnt[h] > 1) {
                sCell[s] = h | DUP;
                hIJK[h] = sIJK[s];
                hM[h] = sM[s];
            }
        }
        // ---- K-means of the purchase orders' points (sum i, sum j)
        const bool on = lane < po;
        int64_t px = 0, py = 0;
        if (on)
            for (uint32_t r = 0; r < per; ++r) {
                const uint32_t p = sIJK[lane * per + r];
                px += ijk_i(p);
                py += ijk_j(p);
            }
        if (on) {
            xy[2 * lane] = static_cast<int32_t>(px);
            xy[2 * lane + 1] = static_cast<int32_t>(py);
        }
        __syncthreads();
        const uint32_t my = wave_kmeans(on, px, py, po, P.k, xy, cen, asg);
        __syncthreads();
        if (lane < WMS_KMAX) {
            int64_t sx = 0, sy = 0, cn = 0;
            for (uint32_t i = 0; i < po; ++i)
                if (asg[i] == lane) {
                    sx += xy[2 * i];
                    sy += xy[2 * i + 1];
                    ++cn;
                }
            cS[3 * lane] = sx;
            cS[3 * lane + 1] = sy;
            cS[3 * lane + 2] = cn;
        }
        __syncthreads();
        // ---- silhouette of the points (distances of mean positions)
        if (on) {
            const int64_t nown = cS[3 * my + 2];
            double si = 0.0;
            if (nown > 1) {
                double a = 0.0;
                for (uint32_t j = 0; j < po; ++j)
                    if (j != lane && asg[j] == my) {
                        const int64_t dx = px - xy[2 * j], dy = py - xy[2 * j + 1];
                        a += std::sqrt(static_cast<double>(dx * dx + dy * dy)) / static_cast<double>(per);
                    }
                a /= static_cast<double>(nown - 1);
                double b = __builtin_inf();
                for (uint32_t c = 0; c < kc; ++c) {
                    const int64_t nc = cS[3 * c + 2];
                    if (c == my || nc == 0) continue;
                    double sum = 0.0;
                    for (uint32_t j = 0; j < po; ++j)
                        if (asg[j] == c) {
                            const int64_t dx = px - xy[2 * j], dy = py - xy[2 * j + 1];
                            sum += std::sqrt(static_cast<double>(dx * dx + dy * dy)) / static_cast<double>(per);
                        }
                    b = std::fmin(b, sum / static_cast<double>(nc));
                }
                if (b != __builtin_inf()) {
                    const double mx = std::fmax(a, b);
                    si = mx == 0.0 ? 0.0 : (b - a) / mx;
                }
            }
            sSil[lane] = si;
        }
        __syncthreads();
        if (lane == 0) {
            double tot = 0.0;
            for (uint32_t i = 0; i < po; ++i) tot += sSil[i];
            P.sil[static_cast<size_t>(run) * P.iters + it] = tot / static_cast<double>(po);
            // area of the triangle of the first three non-empty clusters' centres
            uint32_t live[3], nl = 0;
            for (uint32_t c = 0; c < kc && nl < 3; ++c)
                if (cS[3 * c + 2] > 0) live[nl++] = c;
            double area = 0.0;
            if (nl == 3) {
                const int64_t na = cS[3 * live[0] + 2], nb = cS[3 * live[1] + 2], nc = cS[3 * live[2] + 2];
                const int64_t ax = cS[3 * live[0]], ay = cS[3 * live[0] + 1];
                const int64_t d1x = cS[3 * live[1]] * na - ax * nb, d1y = cS[3 * live[1] + 1] * na - ay * nb;
                const int64_t d2x = cS[3 * live[2]] * na - ax * nc, d2y = cS[3 * live[2] + 1] * na - ay * nc;
                int64_t cr = d1x * d2y - d1y * d2x;
                cr = cr < 0 ? -cr : cr;
                const int64_t den = 2 * static_cast<int64_t>(per) * per * na * na * nb * nc;
                area = static_cast<double>(cr) / static_cast<double>(den);
            }
            P.area[static_cast<size_t>(run) * P.iters + it] = area;
        }
        // ---- the picks, in order
        uint32_t valid = 0, nmov = 0;   // clusters whose cached nearest empty node is current
        for (uint32_t c0 = 0; c0 < S; c0 += 64) {
            const uint32_t s = c0 + lane;
            const bool in = s < S;
            uint32_t rq = 0, rijk = 0, rm = 0, rcell = 0, rart = 0, rc = 0;
            if (in) {
                rq = sQty[s];
                rijk = sIJK[s];
                rm = sM[s];
                rcell = sCell[s];
                rart = sArt[s];
                rc = asg[s / per];
            }
            const uint32_t nl = std::min(64u, S - c0);
            for (uint32_t l = 0; l < nl; ++l) {
                const uint32_t q = __builtin_amdgcn_readlane(rq, l);
                const uint32_t cell = __builtin_amdgcn_readlane(rcell, l);
                const bool dup = cell & DUP;
                const uint32_t hc = cell & ~DUP;
                uint32_t ijk, m;
                if (dup) {
                    ijk = __builtin_amdgcn_readfirstlane(hIJK[hc]);
                    m = __builtin_amdgcn_readfirstlane(hM[hc]);
                } else {
                    ijk = __builtin_amdgcn_readlane(rijk, l);
                    m = __builtin_amdgcn_readlane(rm, l);
                }
                if (m > q) {
                    m -= q;
                } else {
                    const uint32_t c = __builtin_amdgcn_readlane(rc, l);
                    const int64_t sx = cS[3 * c], sy = cS[3 * c + 1], scale = static_cast<int64_t>(per) * cS[3 * c + 2];
                    if (!((valid >> c) & 1u)) {
                        const uint64_t key = nearest_empty<MPW>(mword, nx, ny, sx, sy, scale);
                        best[c] = key;   // every lane writes the same value
                        valid |= 1u << c;
                    }
                    const uint64_t bk = uniform64(best[c]);
                    const uint32_t iv = ijk_i(ijk), jv = ijk_j(ijk), kv = ijk_k(ijk);
                    if (bk != NOKEY && (bk >> 24) < centre_d2(iv, jv, sx, sy, scale)) {
                        // move the article to u; its node v becomes empty
                        const uint32_t u = static_cast<uint32_t>(bk & 0xFFFFFFu);
                        const uint32_t iu = u % nx, tu = u / nx, ju = tu % ny, ku = tu / ny;
                        const uint32_t v = (kv * ny + jv) * nx + iv;
                        const uint32_t ru = ju * nx + iu, rv = jv * nx + iv;
                        // every lane applies the same update to the same words
                        mword[ru / MPW] &= ~rack_bit<MPW>(ru, ku);
                        mword[rv / MPW] |= rack_bit<MPW>(rv, kv);
                        sMov[3 * nmov] = v;
                        sMov[3 * nmov + 1] = u;
                        sMov[3 * nmov + 2] = dup ? hKey[hc] : __builtin_amdgcn_readlane(rart, l);
                        ++nmov;
                        valid &= ~(1u << c);
                        for (uint32_t c2 = 0; c2 < kc; ++c2) {
                            if (!((valid >> c2) & 1u)) continue;
                            const uint64_t b2 = uniform64(best[c2]);
                            if (b2 != NOKEY && static_cast<uint32_t>(b2 & 0xFFFFFFu) == u) {
                                valid &= ~(1u << c2);
                                continue;
                            }
                            const uint64_t kv2 =
                                (centre_d2(iv, jv, cS[3 * c2], cS[3 * c2 + 1],
                                           static_cast<int64_t>(per) * cS[3 * c2 + 2]) << 24) | v;
                            if (kv2 < b2) best[c2] = kv2;
                        }
                        ijk = pack_ijk(iu, ju, ku);
                    }
                    m = P.mmax - (q - m);
                }
                if (dup) {
                    hIJK[hc] = ijk;
                    hM[hc] = m;
                } else if (lane == l) {
                    rijk = ijk;
                    rm = m;
                }
            }
            if (in && !(rcell & DUP)) {
                sIJK[s] = rijk;
                sM[s] = rm;
            }
        }
        __syncthreads();
        // ---- write back: the moves in order, then balances and positions
        if (lane == 0)
            for (uint32_t t = 0; t < nmov; ++t) {
                const uint32_t from = sMov[3 * t], to = sMov[3 * t + 1];
                Ar[from] = 0;
                Mr[from] = 0;
                Ar[to] = sMov[3 * t + 2];
            }
        __syncthreads();
        for (uint32_t s = lane; s < S; s += 64) {
            const uint32_t cell = sCell[s];
            const uint32_t p = (cell & DUP) ? hIJK[cell & ~DUP] : sIJK[s];
            const uint32_t m = (cell & DUP) ? hM[cell & ~DUP] : sM[s];
            const uint32_t v = (ijk_k(p) * ny + ijk_j(p)) * nx + ijk_i(p);
            Mr[v] = m;
            pos[sArt[s]] = v;
        }
        if (lane == 0) P.moves[static_cast<size_t>(run) * P.iters + it] = nmov;
        __syncthreads();
    }
}

uint32_t wms_lds_bytes(uint32_t S, uint32_t H, uint32_t racks, uint32_t mask_bytes) {
    const uint32_t fixed = (3 * WMS_KMAX + 3 * WMS_KMAX + WMS_KMAX + WMS_POMAX) * 8;
    const uint32_t words = 5 * S + 4 * H + 3 * S + 2 * WMS_POMAX + WMS_POMAX;
    return fixed + words * 4 + ((racks * mask_bytes + 3) / 4) * 4;
}

}  // namespace
}  // namespace wr

using namespace wr;

extern "C" wr_status wr_wms_run(wr_context *ctx, const wr_wms_params *p, uint32_t runs, uint32_t iters, uint32_t *A,
                                uint32_t *M, const uint32_t *orders, const uint32_t *qty, double *silhouette,
                                double *area, uint32_t *moves, uint32_t flags, void *stream) {
    WR_API_BEGIN
    if (!ctx) fail(WR_E_INVALID, "context is NULL");
    if (!p) fail(WR_E_INVALID, "params is NULL");
    if (flags & ~static_cast<uint32_t>(WR_DEVICE_PTRS)) fail(WR_E_INVALID, "unknown flags for wr_wms_run");
    const wr_wms_params P = *p;
    if (P.nx < 1 || P.ny < 1 || P.nx > 2048 || P.ny > 2048) fail(WR_E_INVALID, "nx and ny must be in 1..2048");
    if (P.nz < 1 || P.nz > 32) fail(WR_E_INVALID, "nz must be in 1..32");
    const uint64_t racks = static_cast<uint64_t>(P.nx) * P.ny, V = racks * P.nz;
    if (V >= (1u << 24)) fail(WR_E_UNSUPPORTED, "at most 2^24 - 1 nodes");
    const uint32_t mask_bytes = P.nz <= 16 ? 2 : 4;
    if (racks * mask_bytes > WMS_MASK_BYTES)
        fail(WR_E_UNSUPPORTED, "the racks' empty-shelf masks must fit 64 KiB of LDS (nx * ny * " +
                                   std::to_string(mask_bytes) + " bytes)");
    if (P.n_articles < 1 || P.n_articles >= (1u << 24)) fail(WR_E_INVALID, "n_articles must be in 1..2^24-1");
    if (P.mmax < 1 || P.mmax > (1u << 30)) fail(WR_E_INVALID, "mmax must be in 1..2^30");
    if (P.purchase_orders < 1 || P.purchase_orders > WMS_POMAX)
        fail(WR_E_INVALID, "purchase_orders must be in 1..64");
    if (P.articles_per_order < 1) fail(WR_E_INVALID, "articles_per_order must be at least 1");
    const uint64_t S64 = static_cast<uint64_t>(P.purchase_orders) * P.articles_per_order;
    if (S64 > WMS_SMAX) fail(WR_E_UNSUPPORTED, "at most 1024 articles per picking order");
    if (P.clusters < 1 || P.clusters > WMS_KMAX) fail(WR_E_INVALID, "clusters must be in 1..10");
    if (S64 * std::max(P.nx, P.ny) > (1u << 19))
        fail(WR_E_UNSUPPORTED, "articles per order times max(nx, ny) must be at most 2^19 "
                               "(centre distances are compared in 40-bit integers)");
    if (runs == 0 || iters == 0) return WR_OK;
    const uint32_t S = static_cast<uint32_t>(S64);
    uint32_t H = 64;
    while (H < 2 * S) H <<= 1;
    if (!A || !M || !orders || !qty || !silhouette || !area || !moves) fail(WR_E_INVALID, "a buffer is NULL");
    const bool dev = flags & WR_DEVICE_PTRS;
    const uint64_t cells = static_cast<uint64_t>(runs) * V, ocells = static_cast<uint64_t>(runs) * iters * S;
    const uint64_t outs = static_cast<uint64_t>(runs) * iters;
    if (!dev) {
        // the state and the orders are checked here; with device buffers the
        // kernel checks them and the call fails the same way
        std::vector<uint32_t> seen(P.n_articles + 1);
        for (uint32_t r = 0; r < runs; ++r) {
            std::fill(seen.begin(), seen.end(), 0u);
            for (uint64_t v = 0; v < V; ++v) {
                const uint32_t a = A[r * V + v];
                if (a > P.n_articles) fail(WR_E_INVALID, "an article number exceeds n_articles");
                if (a && seen[a]++) fail(WR_E_INVALID, "an article is stored at two nodes");
            }
            for (uint64_t q = 0; q < static_cast<uint64_t>(iters) * S; ++q) {
                const uint64_t o = static_cast<uint64_t>(r) * iters * S + q;
                if (orders[o] < 1 || orders[o] > P.n_articles || !seen[orders[o]])
                    fail(WR_E_INVALID, "an order holds an article that is not stored");
                if (qty[o] > P.mmax) fail(WR_E_RANGE, "a pick takes more than mmax parcels");
            }
        }
    }
    WR_HIP(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (dev) {
        hipEvent_t ev;
        WR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        WR_HIP(hipEventRecord(ev, static_cast<hipStream_t>(stream)));
        WR_HIP(hipStreamWaitEvent(st, ev, 0));
        (void)hipEventDestroy(ev);
    }
    DBuf<uint32_t> d_pos, d_err, d_A, d_M, d_ord, d_qty, d_mov;
    DBuf<double> d_sil, d_area;
    d_pos.alloc(ctx, static_cast<size_t>(runs) * (P.n_articles + 1));
    d_err.alloc(ctx, 1);
    launch_fill_u32(d_err.p, 1, 0u, st);
    WmsArgs a{};
    a.nx = P.nx;
    a.ny = P.ny;
    a.nz = P.nz;
    a.n_articles = P.n_articles;
    a.mmax = P.mmax;
    a.po = P.purchase_orders;
    a.per = P.articles_per_order;
    a.k = P.clusters;
    a.iters = iters;
    a.S = S;
    a.H = H;
    a.pos = d_pos.p;
    a.err = d_err.p;
    if (dev) {
        a.A = A;
        a.M = M;
        a.orders = orders;
        a.qty = qty;
        a.sil = silhouette;
        a.area = area;
        a.moves = moves;
    } else {
        d_A.alloc(ctx, cells);
        d_M.alloc(ctx, cells);
        d_ord.alloc(ctx, ocells);
        d_qty.alloc(ctx, ocells);
        d_sil.alloc(ctx, outs);
        d_area.alloc(ctx, outs);
        d_mov.alloc(ctx, outs);
        WR_HIP(hipMemcpyAsync(d_A.p, A, cells * 4, hipMemcpyHostToDevice, st));
        WR_HIP(hipMemcpyAsync(d_M.p, M, cells * 4, hipMemcpyHostToDevice, st));
        WR_HIP(hipMemcpyAsync(d_ord.p, orders, ocells * 4, hipMemcpyHostToDevice, st));
        WR_HIP(hipMemcpyAsync(d_qty.p, qty, ocells * 4, hipMemcpyHostToDevice, st));
        a.A = d_A.p;
        a.M = d_M.p;
        a.orders = d_ord.p;
        a.qty = d_qty.p;
        a.sil = d_sil.p;
        a.area = d_area.p;
        a.moves = d_mov.p;
    }
    const uint32_t lds = wms_lds_bytes(S, H, static_cast<uint32_t>(racks), mask_bytes);
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (wms)");
    if (mask_bytes == 2)
        hipLaunchKernelGGL(k_wms<2>, runs, 64, lds, st, a);
    else
        hipLaunchKernelGGL(k_wms<1>, runs, 64, lds, st, a);
    check_launch("wms");
    uint32_t err = 0;
    WR_HIP(hipMemcpyAsync(&err, d_err.p, 4, hipMemcpyDeviceToHost, st));
    WR_HIP(hipStreamSynchronize(st));
    if (err & WMS_ERR_STATE) fail(WR_E_INVALID, "a state holds an article number above n_articles or one article at two nodes");
    if (err & WMS_ERR_ORDER)
        fail(WR_E_INVALID, "an order holds an article that is not stored, or a pick of more than mmax parcels");
    if (!dev) {
        WR_HIP(hipMemcpyAsync(A, d_A.p, cells * 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipMemcpyAsync(M, d_M.p, cells * 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipMemcpyAsync(silhouette, d_sil.p, outs * 8, hipMemcpyDeviceToHost, st));
        WR_HIP(hipMemcpyAsync(area, d_area.p, outs * 8, hipMemcpyDeviceToHost, st));
        WR_HIP(hipMemcpyAsync(moves, d_mov.p, outs * 4, hipMemcpyDeviceToHost, st));
        WR_HIP(hipStreamSynchronize(st));
    }
    WR_API_END
}
