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

// squared distance of rack (i, j) to the centre S / scale, times scale^2.
// The call's limits keep scale * i and S below 2^19, so the differences fit
// 32 bits and their squares 38.
__device__ __forceinline__ uint64_t centre_d2(uint32_t i, uint32_t j, int32_t sx, int32_t sy, int32_t scale) {
    const int32_t dx = scale * static_cast<int32_t>(i) - sx, dy = scale * static_cast<int32_t>(j) - sy;
    const uint32_t ax = static_cast<uint32_t>(dx < 0 ? -dx : dx), ay = static_cast<uint32_t>(dy < 0 ? -dy : dy);
    return static_cast<uint64_t>(ax) * ax + static_cast<uint64_t>(ay) * ay;
}

// Empty shelves of rack r: MPW masks of 32 / MPW bits per 4-byte LDS word
// (MPW = 1, 2, 3 for up to 32, 16, 10 shelves).
template <uint32_t MPW>
__device__ __forceinline__ uint32_t rack_mask(const uint32_t *mword, uint32_t r) {
    if constexpr (MPW == 1) return mword[r];
    else return (mword[r / MPW] >> ((32u / MPW) * (r % MPW))) & ((1u << (32u / MPW)) - 1u);
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
__device__ uint64_t nearest_empty(const uint32_t *mword, uint32_t nx, uint32_t ny, int32_t sx, int32_t sy,
                                  int32_t scale, uint32_t &ijk_out) {
    const uint32_t lane = threadIdx.x & 63u;
    const int32_t ci = static_cast<int32_t>(std::min(static_cast<uint32_t>(sx) / static_cast<uint32_t>(scale), nx - 1));
    const int32_t cj = static_cast<int32_t>(std::min(static_cast<uint32_t>(sy) / static_cast<uint32_t>(scale), ny - 1));
    int32_t R = 3;
    for (;;) {
        const int32_t i0 = std::max(ci - R, 0), i1 = std::min(ci + R, static_cast<int32_t>(nx) - 1);
        const int32_t j0 = std::max(cj - R, 0), j1 = std::min(cj + R, static_cast<int32_t>(ny) - 1);
        uint64_t best = NOKEY;
        uint32_t bijk = 0;
        for (int32_t jb = j0; jb <= j1; jb += 8)
            for (int32_t ib = i0; ib <= i1; ib += 8) {
                const int32_t i = ib + static_cast<int32_t>(lane & 7u), j = jb + static_cast<int32_t>(lane >> 3);
                if (i <= i1 && j <= j1) {
                    const uint32_t mk = rack_mask<MPW>(mword, static_cast<uint32_t>(j) * nx + static_cast<uint32_t>(i));
                    if (mk) {
                        const uint32_t k = __builtin_ctz(mk);
                        const uint32_t node = (k * ny + static_cast<uint32_t>(j)) * nx + static_cast<uint32_t>(i);
                        const uint64_t key = (centre_d2(i, j, sx, sy, scale) << 24) | node;
                        if (key < best) {
                            best = key;
                            bijk = pack_ijk(static_cast<uint32_t>(i), static_cast<uint32_t>(j), k);
                        }
                    }
                }
            }
        const uint64_t mine = best;
        best = wave_min_u64(best);
        // nearest any rack outside the window can be (the centre lies in
        // the window's column and row ranges)
        uint64_t lb = NOKEY;
        if (i0 > 0) {
            const uint64_t d = static_cast<uint32_t>(sx - scale * (i0 - 1));
            lb = std::min(lb, d * d);
        }
        if (i1 < static_cast<int32_t>(nx) - 1) {
            const uint64_t d = static_cast<uint32_t>(scale * (i1 + 1) - sx);
            lb = std::min(lb, d * d);
        }
        if (j0 > 0) {
            const uint64_t d = static_cast<uint32_t>(sy - scale * (j0 - 1));
            lb = std::min(lb, d * d);
        }
        if (j1 < static_cast<int32_t>(ny) - 1) {
            const uint64_t d = static_cast<uint32_t>(scale * (j1 + 1) - sy);
            lb = std::min(lb, d * d);
        }
        if (lb == NOKEY || (best != NOKEY && (best >> 24) < lb)) {
            const uint64_t won = __builtin_amdgcn_ballot_w64(mine == best && best != NOKEY);
            ijk_out = won ? __builtin_amdgcn_readlane(bijk, static_cast<uint32_t>(__builtin_ctzll(won))) : 0u;
            return best;
        }
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
    uint64_t *best = reinterpret_cast<uint64_t *>(cen + 3 * WMS_KMAX);   // [KMAX] nearest empty key
    double *sSil = reinterpret_cast<double *>(best + WMS_KMAX);          // [POMAX]
    uint32_t *sArt = reinterpret_cast<uint32_t *>(sSil + WMS_POMAX);     // [S]
    uint32_t *sQty = sArt + S, *sIJK = sQty + S, *sM = sIJK + S, *sCell = sM + S;
    // hash cells of the order's articles: key (bit 31 = picked more than
    // once), and the live node and balance of a repeated article
    uint32_t *hKey = sCell + S, *hIJK = hKey + H, *hM = hIJK + H;
    int32_t *xy = reinterpret_cast<int32_t *>(hM + H);   // [2 POMAX]
    uint32_t *asg = reinterpret_cast<uint32_t *>(xy + 2 * WMS_POMAX);   // [POMAX]
    int32_t *cS = reinterpret_cast<int32_t *>(asg + WMS_POMAX);   // [3 KMAX] sum x, sum y, count per cluster
    uint32_t *mword = reinterpret_cast<uint32_t *>(cS + 3 * WMS_KMAX);   // rack masks, MPW per 4-byte word
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
#pragma unroll 4
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
#pragma unroll 4
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
        for (uint32_t h = lane; h < H; h += 64) hKey[h] = 0;
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
            // linear probing; H > S cells always leave one free
            uint32_t h = (a * 2654435761u) & (H - 1);
            for (;;) {
                const uint32_t old = atomicCAS(&hKey[h], 0u, a);
                if (old == 0u) break;
                if ((old & ~DUP) == a) {
                    atomicOr(&hKey[h], DUP);
                    break;
                }
                h = (h + 1) & (H - 1);
            }
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
            if (hKey[h] & DUP) {
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
            int32_t sx = 0, sy = 0, cn = 0;
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
        // ---- silhouette of the points (distances of mean positions): one
        // distance per pair, summed per cluster in ascending point order
        const int32_t px32 = static_cast<int32_t>(px), py32 = static_cast<int32_t>(py);
        {
            double acc[WMS_KMAX];
#pragma unroll
            for (uint32_t c = 0; c < WMS_KMAX; ++c) acc[c] = 0.0;
            for (uint32_t j = 0; j < po; ++j) {
                const int64_t dx = px - __builtin_amdgcn_readlane(px32, j);
                const int64_t dy = py - __builtin_amdgcn_readlane(py32, j);
                const double d = std::sqrt(static_cast<double>(dx * dx + dy * dy)) / static_cast<double>(per);
                const uint32_t cj = __builtin_amdgcn_readlane(my, j);
#pragma unroll
                for (uint32_t c = 0; c < WMS_KMAX; ++c)
                    if (c < kc && c == cj) acc[c] += d;   // d(i, i) = 0 adds nothing
            }
            if (on) {
                const int32_t nown = cS[3 * my + 2];
                double si = 0.0, a = 0.0, b = __builtin_inf();
#pragma unroll
                for (uint32_t c = 0; c < WMS_KMAX; ++c) {
                    if (c >= kc) continue;
                    const int32_t nc = cS[3 * c + 2];
                    if (c == my) a = acc[c] / static_cast<double>(nown - 1);
                    else if (nc > 0) b = std::fmin(b, acc[c] / static_cast<double>(nc));
                }
                if (nown > 1 && b != __builtin_inf()) {
                    const double mx = std::fmax(a, b);
                    si = mx == 0.0 ? 0.0 : (b - a) / mx;
                }
                sSil[lane] = si;
            }
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
        // ---- the picks, in order.  A chunk of 64 slots is evaluated at once
        // against the state as it stands; the first slot that would change
        // shared state (a move), needs a nearest-empty search, or picks an
        // article picked earlier in the order ends the chunk's final prefix
        // and runs alone; then the rest of the chunk is evaluated again.
        uint32_t valid = 0, nmov = 0;   // clusters whose cached nearest empty node is current
        // cluster c's centre and cached nearest empty node live in lane c
        int32_t cl_sx = 0, cl_sy = 0, cl_scale = 1;
        uint64_t cl_best = NOKEY;
        uint32_t cl_bijk = 0;
        if (lane < kc) {
            cl_sx = cS[3 * lane];
            cl_sy = cS[3 * lane + 1];
            cl_scale = static_cast<int32_t>(per) * cS[3 * lane + 2];
        }
        for (uint32_t c0 = 0; c0 < S; c0 += 64) {
            const uint32_t s = c0 + lane;
            const uint32_t nl = std::min(64u, S - c0);
            const bool in = lane < nl;
            uint32_t rq = 0, rijk = 0, rm = 0, rcell = 0, rart = 0, rc = 0;
            uint64_t rdv = 0;   // the slot node's distance to its cluster's centre
            if (in) {
                rq = sQty[s];
                rijk = sIJK[s];
                rm = sM[s];
                rcell = sCell[s];
                rart = sArt[s];
                rc = asg[s / per];
                rdv = centre_d2(ijk_i(rijk), ijk_j(rijk), cS[3 * rc], cS[3 * rc + 1],
                                static_cast<int32_t>(per) * cS[3 * rc + 2]);
            }
            uint32_t start = 0;
            for (;;) {
                // nearest-empty searches for the clusters the remaining
                // restocks need (each serves at least its first one)
                const bool restock = in && lane >= start && !(rcell & DUP) && rm <= rq;
                for (uint32_t c = 0; c < kc; ++c) {
                    if ((valid >> c) & 1u) continue;
                    if (!__builtin_amdgcn_ballot_w64(restock && rc == c)) continue;
                    uint32_t bij = 0;
                    const int32_t sx = __builtin_amdgcn_readlane(cl_sx, c), sy = __builtin_amdgcn_readlane(cl_sy, c);
                    const uint64_t key =
                        nearest_empty<MPW>(mword, nx, ny, sx, sy, __builtin_amdgcn_readlane(cl_scale, c), bij);
                    if (lane == c) {
                        cl_best = key;
                        cl_bijk = bij;
                        best[c] = key;
                    }
                    valid |= 1u << c;
                }
                __builtin_amdgcn_wave_barrier();   // lane c's best[c] before the other lanes read it
                bool stop = false;
                uint32_t nm = rm;
                if (in && lane >= start) {
                    if (rcell & DUP) {
                        stop = true;
                    } else if (rm > rq) {
                        nm = rm - rq;
                    } else {
                        const uint64_t bk = best[rc];
                        if (bk != NOKEY && (bk >> 24) < rdv) stop = true;
                        else nm = P.mmax - (rq - rm);
                    }
                }
                const uint64_t sm = __builtin_amdgcn_ballot_w64(stop);
                const uint32_t l = sm ? static_cast<uint32_t>(__builtin_ctzll(sm)) : nl;
                if (in && lane >= start && lane < l) rm = nm;   // the final prefix
                if (l >= nl) break;
                // ---- slot l alone
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
                    const int32_t sx = __builtin_amdgcn_readlane(cl_sx, c), sy = __builtin_amdgcn_readlane(cl_sy, c);
                    const int32_t scale = __builtin_amdgcn_readlane(cl_scale, c);
                    if (!((valid >> c) & 1u)) {
                        uint32_t bij = 0;
                        const uint64_t key = nearest_empty<MPW>(mword, nx, ny, sx, sy, scale, bij);
                        if (lane == c) {
                            cl_best = key;
                            cl_bijk = bij;
                            best[c] = key;
                        }
                        valid |= 1u << c;
                    }
                    const uint64_t bk = readlane64(cl_best, c);
                    const uint32_t iv = ijk_i(ijk), jv = ijk_j(ijk), kv = ijk_k(ijk);
                    if (bk != NOKEY && (bk >> 24) < centre_d2(iv, jv, sx, sy, scale)) {
                        // move the article to u; its node v becomes empty
                        const uint32_t u = static_cast<uint32_t>(bk & 0xFFFFFFu);
                        const uint32_t uijk = __builtin_amdgcn_readlane(cl_bijk, c);
                        const uint32_t iu = ijk_i(uijk), ju = ijk_j(uijk), ku = ijk_k(uijk);
                        const uint32_t v = (kv * ny + jv) * nx + iv;
                        const uint32_t ru = ju * nx + iu, rv = jv * nx + iv;
                        // every lane applies the same update to the same words
                        mword[ru / MPW] &= ~rack_bit<MPW>(ru, ku);
                        mword[rv / MPW] |= rack_bit<MPW>(rv, kv);
                        // the state in HBM, in move order from one lane; the
                        // final balances follow after the picks
                        const uint32_t art = dup ? (hKey[hc] & ~DUP) : __builtin_amdgcn_readlane(rart, l);
                        if (lane == 0) {
                            Ar[v] = 0;
                            Mr[v] = 0;
                            Ar[u] = art;
                        }
                        ++nmov;
                        // the caches: cluster c's node is taken; every other
                        // cluster drops u, or takes v when v is nearer
                        bool drop = false;
                        if (lane < kc && lane != c && ((valid >> lane) & 1u)) {
                            if (cl_best != NOKEY && static_cast<uint32_t>(cl_best & 0xFFFFFFu) == u) {
                                drop = true;
                            } else {
                                const uint64_t kv2 = (centre_d2(iv, jv, cl_sx, cl_sy, cl_scale) << 24) | v;
                                if (kv2 < cl_best) {
                                    cl_best = kv2;
                                    cl_bijk = ijk;
                                    best[lane] = kv2;
                                }
                            }
                        }
                        valid &= ~static_cast<uint32_t>(__builtin_amdgcn_ballot_w64(drop)) & ~(1u << c);
                        ijk = uijk;
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
                start = l + 1;
            }
            if (in && !(rcell & DUP)) {
                sIJK[s] = rijk;
                sM[s] = rm;
            }
        }
        __syncthreads();
        // ---- write back: balances and positions (after the moves' stores)
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

uint32_t wms_lds_bytes(uint32_t S, uint32_t H, uint32_t mask_words) {
    const uint32_t fixed = (3 * WMS_KMAX + WMS_KMAX + WMS_POMAX) * 8;
    const uint32_t words = 5 * S + 3 * H + 2 * WMS_POMAX + WMS_POMAX + 3 * WMS_KMAX;
    return fixed + (words + mask_words) * 4;
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
    // racks per 4-byte mask word: three of 10 bits, two of 16, or one
    const uint32_t mpw = P.nz <= 10 ? 3 : (P.nz <= 16 ? 2 : 1);
    const uint64_t mask_words = (racks + mpw - 1) / mpw;
    if (mask_words * 4 > WMS_MASK_BYTES)
        fail(WR_E_UNSUPPORTED, "the racks' empty-shelf masks must fit 64 KiB of LDS (" +
                                   std::to_string(mpw) + " racks per 4 bytes)");
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
    while (H <= S) H <<= 1;
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
    const uint32_t lds = wms_lds_bytes(S, H, static_cast<uint32_t>(mask_words));
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (wms)");
    if (mpw == 3)
        hipLaunchKernelGGL(k_wms<3>, runs, 64, lds, st, a);
    else if (mpw == 2)
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
