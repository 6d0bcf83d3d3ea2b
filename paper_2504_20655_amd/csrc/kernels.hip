// gfx950 kernels of the routing hot path.
//
// Every kernel computes a piece of the min-plus relaxation
//     d(v) <- min(d(v), d(u) + w(u, v))   for arcs (u, v)
// that Bellman-Ford iterates to its unique fixpoint on graphs with
// non-negative weights (GPU Implementation subsection of the paper), or
// reads the fixpoint out (order matrices, predecessors).  Distances are
// uint32 with WR_INF = 0xFFFFFFFF; candidate sums use a saturating add, so
// INF + w stays INF and no candidate wraps.
//
// Wave64 is assumed throughout (CDNA).  Values a whole wave agrees on are
// passed through readfirstlane so that the compiler keeps them in SGPRs and
// loads CSR rows through the scalar cache.
#include "kmeans_wave.hpp"
#include "wr_internal.hpp"

namespace wr {

namespace {

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    return __builtin_elementwise_add_sat(a, b);
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t uniform(uint32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}

// number of set bits of `mask` below this lane
__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask) {
    uint32_t lo = __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u);
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32), lo);
}

inline uint32_t blocks_for(size_t n, uint32_t threads, uint32_t cap = 65535u * 4u) {
    size_t b = (n + threads - 1) / threads;
    if (b == 0) b = 1;
    if (b > cap) b = cap;
    return static_cast<uint32_t>(b);
}

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
    size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
    size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    const size_t n4 = n / 4;
    uint4 *p4 = reinterpret_cast<uint4 *>(p);
    const uint4 v4 = make_uint4(v, v, v, v);
    for (size_t k = i; k < n4; k += stride) p4[k] = v4;
    for (size_t k = n4 * 4 + i; k < n; k += stride) p[k] = v;
}

__global__ void k_fill_u32_unaligned(uint32_t *__restrict__ p, size_t n, uint32_t v) {
    size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
    size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t k = i; k < n; k += stride) p[k] = v;
}

__global__ void k_fill_u8(uint8_t *__restrict__ p, size_t n, uint8_t v) {
    size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
    size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t k = i; k < n; k += stride) p[k] = v;
}

// --------------------------------------------------- blocked layout kernels
// dist[b][v][l]: source 64*b + l of the chunk, vertex v; one wave covers the
// 64 sources of a block at one vertex, so every access is a 256-byte line.
__global__ void k_blk_seed(uint32_t *__restrict__ dist, uint32_t V, uint32_t S,
                           const uint32_t *__restrict__ src) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    size_t b = i / LANES, l = i % LANES;
    dist[(b * V + src[i]) * LANES + l] = 0;
}

// Pull sweep, in place: d(v) <- min(d(v), min over in-arcs (u,v) of d(u)+w).
// One wave per (block, vertex) unit, lanes = sources.  Any order of these
// updates converges to the same fixpoint; `changed` is set if a value moved.
__global__ __launch_bounds__(256) void k_sweep_pull(uint32_t *__restrict__ dist, uint32_t V,
                                                    uint32_t nb,
                                                    const uint32_t *__restrict__ in_ptr,
                                                    const uint32_t *__restrict__ in_src,
                                                    const uint32_t *__restrict__ in_w,
                                                    uint32_t *__restrict__ changed) {
    const uint32_t lane = lane_id();
    const uint64_t wave = uniform(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / 64);
    const uint64_t units = static_cast<uint64_t>(nb) * V;
    bool moved = false;
    for (uint64_t u = wave; u < units; u += nwaves) {
        const uint32_t b = static_cast<uint32_t>(u / V);
        const uint32_t v = static_cast<uint32_t>(u - static_cast<uint64_t>(b) * V);
        const uint32_t beg = uniform(in_ptr[v]), end = uniform(in_ptr[v + 1]);
        if (beg == end) continue;
        uint32_t *db = dist + static_cast<size_t>(b) * V * LANES;
        const uint32_t old = db[static_cast<size_t>(v) * LANES + lane];
        uint32_t m = old;
        for (uint32_t e = beg; e < end; ++e) {
            const uint32_t x = uniform(in_src[e]);
            const uint32_t ww = uniform(in_w[e]);
            m = min(m, sat_add(db[static_cast<size_t>(x) * LANES + lane], ww));
        }
        if (m < old) {
            db[static_cast<size_t>(v) * LANES + lane] = m;
            moved = true;
        }
    }
    if (moved) *changed = 1u;
}

__global__ void k_frontier_seed(uint64_t *__restrict__ list, uint32_t *__restrict__ count,
                                uint32_t S, const uint32_t *__restrict__ src) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S) list[i] = (static_cast<uint64_t>(i / LANES) << 32) | src[i];
    if (i == 0) *count = S;
}

// Push relaxation of the frontier items (block, v): each lane (source)
// relaxes every out-arc of v; an arc target whose value dropped for any lane
// is queued once for the next pass (a 32-bit pass stamp per (block, vertex)
// dedups).  The wave collects its item's improved targets one per lane,
// stamps them in parallel, and reserves the queue slots of the winners with
// one atomic (their offsets from mbcnt).
__global__ __launch_bounds__(256) void k_frontier_push(
    uint32_t *__restrict__ dist, uint32_t V, const uint32_t *__restrict__ row_ptr,
    const uint32_t *__restrict__ col, const uint32_t *__restrict__ w,
    const uint64_t *__restrict__ list_in, const uint32_t *__restrict__ count_in,
    uint64_t *__restrict__ list_out, uint32_t *__restrict__ count_out,
    uint32_t *__restrict__ stamps, const uint32_t *__restrict__ pass_ctr) {
    const uint32_t lane = lane_id();
    const uint32_t wave = uniform(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
    const uint32_t nwaves = gridDim.x * (blockDim.x / 64);
    const uint32_t n = uniform(*count_in);
    const uint32_t stamp = uniform(*pass_ctr) + 1u;
    for (uint32_t i = wave; i < n; i += nwaves) {
        const uint64_t item = list_in[i];
        const uint32_t b = uniform(static_cast<uint32_t>(item >> 32));
        const uint32_t v = uniform(static_cast<uint32_t>(item));
        uint32_t *db = dist + static_cast<size_t>(b) * V * LANES;
        const uint32_t dv = db[static_cast<size_t>(v) * LANES + lane];
        const uint32_t beg = uniform(row_ptr[v]), end = uniform(row_ptr[v + 1]);
        uint32_t tgt = 0, nq = 0;   // lane k < nq holds the k-th improved target
        for (uint32_t e = beg; e < end; ++e) {
            const uint32_t x = uniform(col[e]);
            const uint32_t nd = sat_add(dv, uniform(w[e]));
            uint32_t *px = db + static_cast<size_t>(x) * LANES + lane;
            bool imp = false;
            if (nd < *px) imp = nd < atomicMin(px, nd);
            if (__builtin_amdgcn_ballot_w64(imp) != 0) {
                if (lane == nq) tgt = x;
                ++nq;
            }
            if (nq == LANES || (e + 1 == end && nq)) {
                bool win = false;
                if (lane < nq) win = atomicMax(&stamps[static_cast<size_t>(b) * V + tgt], stamp) < stamp;
                const uint64_t wm = __builtin_amdgcn_ballot_w64(win);
                uint32_t base = 0;
                if (lane == 0 && wm) base = atomicAdd(count_out, static_cast<uint32_t>(__builtin_popcountll(wm)));
                base = uniform(base);
                if (win) list_out[base + mbcnt64(wm)] = (static_cast<uint64_t>(b) << 32) | tgt;
                nq = 0;
            }
        }
    }
}

// out[r][v] = dist of chunk source row_src_idx[r] at v (source-major rows).
__global__ void k_blk_emit(const uint32_t *__restrict__ dist, uint32_t V, uint32_t rows,
                           const uint32_t *__restrict__ row_src_idx,
                           const uint32_t *__restrict__ out_row, uint32_t *__restrict__ out) {
    for (uint32_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const uint32_t idx = row_src_idx[r];
        const size_t b = idx / LANES, l = idx % LANES;
        const uint32_t *db = dist + b * V * LANES;
        uint32_t *o = out + static_cast<size_t>(out_row[r]) * V;
        for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x)
            o[v] = db[static_cast<size_t>(v) * LANES + l];
    }
}

__global__ void k_pass_prologue(uint32_t *__restrict__ count_next,
                                const uint32_t *__restrict__ count_cur,
                                unsigned long long *__restrict__ stats,
                                uint32_t *__restrict__ pass_ctr) {
    const uint32_t c = *count_cur;
    stats[0] += c;
    stats[1] += c ? 1ull : 0ull;
    *count_next = 0;
    *pass_ctr += 1u;
}

// ------------------------------------------------------ segmented schedule
// Work state of one chunk of S sources over T tiles (see TileSet):
//   gdist[s][Vt]   full distance state, written at a tile's first visit
//   inbox[s][NP]   values pushed into boundary-in vertices by other tiles
//   visited[s][T]  whether gdist of (s, t) has been written
//   stamps[s][T]   pass stamp of the last activation (dedup)
//   bucket[par][t][k], cnt[par][t]   sources active in tile t for a pass
//   tiles[par][j], ntiles[par]       tiles with a non-empty bucket
//   units[u] = (tile, slice)         slices of G sources, built per pass
struct SegPassArgs {
    // tables
    const uint32_t *tile_base, *l_off, *l_arc, *x_off, *x_port, *x_w, *x_tile, *port_base,
        *port_local, *bo_base, *bo_local;
    uint32_t T, Vt, NP;
    // state
    uint32_t S;
    uint32_t *gdist, *inbox;
    uint8_t *visited;
    uint32_t *stamps;
    const uint32_t *src_pos, *src_tile;
    // activation buffers (current / next parity)
    const uint32_t *cnt_cur, *bucket_cur;
    uint32_t *cnt_next, *bucket_next, *tiles_next, *ntiles_next;
    const uint2 *units;
    const uint32_t *nunits;
    uint32_t *cursor;
    const uint32_t *pass_ctr;
    uint32_t G;
    // source-blocked schedule: in-tile in-arcs and the sources of the chunk
    const uint32_t *li_off, *li_arc;
    uint32_t nsrc;
    // overlay schedule: activation flags [T][S] instead of stamped lists;
    // per block the value of every exit, xval[S][NB][64]; per port p its
    // incoming cross arcs k in [pin_off[p], pin_off[p+1]) with their records
    // pin_rec[k] = {source exit, w | local port << 16}; per tile {first
    // incoming arc, incoming arcs} in hdr2
    uint8_t *flags;
    uint32_t *xval;
    uint32_t NB;
    const uint32_t *pin_off;
    const uint2 *pin_rec;
    const uint2 *hdr2;
    // overlay work counters, each entry owned by one wave (no atomics):
    // visits of each tile, and exit values stored per (workgroup, wave)
    uint32_t *tile_visits;
    uint32_t *wave_stores;
    // target-bounded passes: per source slot (block * 64 + lane) the largest
    // value worth storing, or NULL (no bound)
    const uint32_t *bound;
};

__device__ __forceinline__ void seg_activate(const SegPassArgs &A, uint32_t s, uint32_t t,
                                             uint32_t stamp) {
    if (A.flags) {
        A.flags[static_cast<size_t>(t) * A.S + s] = 1;
        return;
    }
    const uint32_t o = atomicMax(&A.stamps[static_cast<size_t>(s) * A.T + t], stamp);
    if (o < stamp) {
        const uint32_t k = atomicAdd(&A.cnt_next[t], 1u);
        A.bucket_next[static_cast<size_t>(t) * A.S + k] = s;
        if (k == 0) {
            const uint32_t j = atomicAdd(A.ntiles_next, 1u);
            A.tiles_next[j] = t;
        }
    }
}

// One pass over the active (tile, source) items.  A workgroup takes one
// unit (a tile and up to G of its active sources), stages the tile's
// in-tile arcs in LDS once, and its NW waves each relax one source of the
// unit at a time: the tile's distances for that source live in the wave's
// own LDS array, and a FIFO of changed vertices (deduplicated by a bitmap)
// drives push relaxation until the tile reaches its local fixpoint.  Changed
// values are written back, and every changed boundary-out vertex pushes its
// cross-tile arcs into the target tile's inbox with atomicMin, activating
// (source, target tile) for the next pass when the inbox value dropped.
template <int CAP, int NW>
__global__ __launch_bounds__(NW * 64) void k_seg_pass(SegPassArgs A) {
    constexpr uint32_t ARC_CAP = 4u * CAP;
    constexpr uint32_t WORDS = CAP / 32;
    __shared__ uint16_t s_off[CAP + 2];
    __shared__ uint32_t s_arc[ARC_CAP];
    __shared__ uint32_t s_dist[NW][CAP];
    __shared__ uint16_t s_q[NW][CAP];
    __shared__ uint32_t s_inq[NW][WORDS];
    __shared__ uint32_t s_dirty[NW][WORDS];
    __shared__ uint32_t s_unit;

    const uint32_t lane = lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    const uint32_t nunits = uniform(*A.nunits);
    const uint32_t stamp = uniform(*A.pass_ctr) + 1u;
    uint32_t *dist = s_dist[wv];
    uint16_t *q = s_q[wv];
    uint32_t *inq = s_inq[wv];
    uint32_t *dirty = s_dirty[wv];
    uint32_t staged = NONE;

    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(A.cursor, 1u);
        __syncthreads();
        const uint32_t u = uniform(s_unit);
        __syncthreads();
        if (u >= nunits) break;
        const uint2 unit = A.units[u];
        const uint32_t t = uniform(unit.x), slice = uniform(unit.y);
        const uint32_t base = uniform(A.tile_base[t]);
        const uint32_t n = uniform(A.tile_base[t + 1]) - base;
        if (t != staged) {
            const uint32_t a0 = A.l_off[base];
            for (uint32_t i = threadIdx.x; i <= n; i += blockDim.x)
                s_off[i] = static_cast<uint16_t>(A.l_off[base + i] - a0);
            const uint32_t na = A.l_off[base + n] - a0;
            for (uint32_t i = threadIdx.x; i < na; i += blockDim.x) s_arc[i] = A.l_arc[a0 + i];
            staged = t;
            __syncthreads();
        }
        const uint32_t total = uniform(A.cnt_cur[t]);
        const uint32_t first_k = slice * A.G;
        const uint32_t cnt = min(A.G, total - first_k);
        for (uint32_t k = wv; k < cnt; k += NW) {
            const uint32_t s = uniform(A.bucket_cur[static_cast<size_t>(t) * A.S + first_k + k]);
            const size_t st = static_cast<size_t>(s) * A.T + t;
            const bool first = A.visited[st] == 0;
            uint32_t *gd = A.gdist + static_cast<size_t>(s) * A.Vt + base;
            for (uint32_t i = lane; i < n; i += 64) dist[i] = first ? INF : gd[i];
            for (uint32_t i = lane; i < WORDS; i += 64) {
                inq[i] = 0;
                dirty[i] = 0;
            }
            __builtin_amdgcn_wave_barrier();
            uint32_t head = 0, tail = 0;
            // seed: the source itself
            if (uniform(A.src_tile[s]) == t) {
                const uint32_t loc = uniform(A.src_pos[s]) - base;
                // decide once for the wave before lane 0 writes the value
                const bool need = uniform(dist[loc]) != 0;
                __builtin_amdgcn_wave_barrier();
                if (need) {
                    if (lane == 0) {
                        dist[loc] = 0;
                        inq[loc >> 5] |= 1u << (loc & 31);
                        dirty[loc >> 5] |= 1u << (loc & 31);
                        q[0] = static_cast<uint16_t>(loc);
                    }
                    tail = 1;
                }
            }
            __builtin_amdgcn_wave_barrier();
            // seed: boundary-in vertices whose inbox value beats the stored one
            const uint32_t p0 = uniform(A.port_base[t]), p1 = uniform(A.port_base[t + 1]);
            const uint32_t *ib = A.inbox + static_cast<size_t>(s) * A.NP;
            for (uint32_t kk = p0; kk < p1; kk += 64) {
                const uint32_t k2 = kk + lane;
                bool push = false;
                uint32_t loc = 0;
                if (k2 < p1) {
                    loc = A.port_local[k2];
                    const uint32_t v = ib[k2];
                    if (v < dist[loc]) {
                        dist[loc] = v;
                        atomicOr(&dirty[loc >> 5], 1u << (loc & 31));
                        const uint32_t ob = atomicOr(&inq[loc >> 5], 1u << (loc & 31));
                        push = (ob & (1u << (loc & 31))) == 0;
                    }
                }
                const uint64_t m = __builtin_amdgcn_ballot_w64(push);
                if (push) q[(tail + mbcnt64(m)) & (CAP - 1)] = static_cast<uint16_t>(loc);
                tail += __builtin_popcountll(m);
                __builtin_amdgcn_wave_barrier();
            }
            // relax to the local fixpoint
            while (head != tail) {
                const uint32_t avail = tail - head;
                const uint32_t take = avail < 64 ? avail : 64;
                const bool act = lane < take;
                uint32_t x0 = 0, du = INF, e = 0, e_end = 0;
                if (act) {
                    x0 = q[(head + lane) & (CAP - 1)];
                    atomicAnd(&inq[x0 >> 5], ~(1u << (x0 & 31)));
                }
                __builtin_amdgcn_wave_barrier();
                if (act) {
                    du = __hip_atomic_load(&dist[x0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    e = s_off[x0];
                    e_end = s_off[x0 + 1];
                }
                head += take;
                while (__builtin_amdgcn_ballot_w64(e < e_end) != 0) {
                    bool newq = false;
                    uint32_t x = 0;
                    if (e < e_end) {
                        const uint32_t a = s_arc[e];
                        ++e;
                        x = a >> 16;
                        const uint32_t nd = sat_add(du, a & 0xFFFFu);
                        const uint32_t old = atomicMin(&dist[x], nd);
                        if (nd < old) {
                            const uint32_t bit = 1u << (x & 31);
                            atomicOr(&dirty[x >> 5], bit);
                            newq = (atomicOr(&inq[x >> 5], bit) & bit) == 0;
                        }
                    }
                    const uint64_t m = __builtin_amdgcn_ballot_w64(newq);
                    if (newq) q[(tail + mbcnt64(m)) & (CAP - 1)] = static_cast<uint16_t>(x);
                    tail += __builtin_popcountll(m);
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __builtin_amdgcn_wave_barrier();
            // write back: everything on the first visit, changed values after
            for (uint32_t i = lane; i < n; i += 64) {
                const bool d = first || ((dirty[i >> 5] >> (i & 31)) & 1u);
                if (d) gd[i] = dist[i];
            }
            if (lane == 0 && first) A.visited[st] = 1;
            // boundary exchange: push changed boundary-out vertices across tiles
            const uint32_t b0 = uniform(A.bo_base[t]), b1 = uniform(A.bo_base[t + 1]);
            uint32_t *ibox = A.inbox + static_cast<size_t>(s) * A.NP;
            for (uint32_t kk = b0 + lane; kk < b1; kk += 64) {
                const uint32_t loc = A.bo_local[kk];
                if (!((dirty[loc >> 5] >> (loc & 31)) & 1u)) continue;
                const uint32_t dv = dist[loc];
                const uint32_t pos = base + loc;
                const uint32_t xe1 = A.x_off[pos + 1];
                for (uint32_t xe = A.x_off[pos]; xe < xe1; ++xe) {
                    const uint32_t nd = sat_add(dv, A.x_w[xe]);
                    uint32_t *pi = ibox + A.x_port[xe];
                    if (nd < *pi && nd < atomicMin(pi, nd)) seg_activate(A, s, A.x_tile[xe], stamp);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

// Wave 0 turns the set bits of bitmap bm[WORDS] (WORDS <= 64) into list[]
// (ascending) and stores the count in *len; with clear, the bitmap is
// zeroed on the way.  The exclusive prefix of the per-word counts is built
// from readlane broadcasts (uniform loop over the words).
template <uint32_t WORDS>
__device__ __forceinline__ void compact_bits(uint32_t *bm, uint16_t *list, uint32_t *len, bool clear) {
    static_assert(WORDS <= 64, "one word per lane");
    const uint32_t lane = lane_id();
    const bool in = lane < WORDS;
    uint32_t word = in ? bm[lane] : 0u;
    if (in && clear) bm[lane] = 0u;
    const uint32_t c = __builtin_popcount(word);
    uint32_t excl = 0, total = 0;
#pragma unroll
    for (uint32_t k = 0; k < WORDS; ++k) {
        const uint32_t ck = __builtin_amdgcn_readlane(c, k);
        excl += lane > k ? ck : 0u;
        total += ck;
    }
    uint32_t pos = excl;
    while (word) {
        const uint32_t j = __builtin_ctz(word);
        word &= word - 1u;
        list[pos++] = static_cast<uint16_t>(lane * 32 + j);
    }
    if (lane == 0) *len = total;
}

// Pull update of candidate v for the 64 lanes: returns whether any lane
// improved.  The in-arcs of v are read across lanes in one LDS access and
// broadcast with readlane, so the row reads D[u] of all arcs are independent.
template <int CAP>
__device__ __forceinline__ bool pull_row(uint32_t *D, const uint32_t *s_iinfo, const uint32_t *s_iarc,
                                        uint32_t v, uint32_t lane) {
    const uint32_t info = uniform(s_iinfo[v]);
    const uint32_t off = info >> 16, deg = info & 0xFFFFu;
    const uint32_t old = D[v * 64 + lane];
    uint32_t m = old;
    for (uint32_t c0 = 0; c0 < deg; c0 += 64) {
        const uint32_t mine = c0 + lane < deg ? s_iarc[off + c0 + lane] : 0u;
        const uint32_t nk = deg - c0 < 64 ? deg - c0 : 64;
        uint32_t k = 0;
        for (; k + 4 <= nk; k += 4) {
            const uint32_t a0 = __builtin_amdgcn_readlane(mine, k);
            const uint32_t a1 = __builtin_amdgcn_readlane(mine, k + 1);
            const uint32_t a2 = __builtin_amdgcn_readlane(mine, k + 2);
            const uint32_t a3 = __builtin_amdgcn_readlane(mine, k + 3);
            const uint32_t d0 = D[(a0 >> 16) * 64 + lane], d1 = D[(a1 >> 16) * 64 + lane];
            const uint32_t d2 = D[(a2 >> 16) * 64 + lane], d3 = D[(a3 >> 16) * 64 + lane];
            m = min(m, min(min(sat_add(d0, a0 & 0xFFFFu), sat_add(d1, a1 & 0xFFFFu)),
                           min(sat_add(d2, a2 & 0xFFFFu), sat_add(d3, a3 & 0xFFFFu))));
        }
        for (; k < nk; ++k) {
            const uint32_t a = __builtin_amdgcn_readlane(mine, k);
            m = min(m, sat_add(D[(a >> 16) * 64 + lane], a & 0xFFFFu));
        }
    }
    const bool imp = m < old;
    if (imp) D[v * 64 + lane] = m;
    return __builtin_amdgcn_ballot_w64(imp) != 0;
}

// Marks the in-tile out-neighbours of v in bitmap bm (lanes take one arc each).
__device__ __forceinline__ void mark_out(uint32_t *bm, const uint32_t *s_oinfo, const uint16_t *s_odst,
                                         uint32_t v, uint32_t lane) {
    const uint32_t info = uniform(s_oinfo[v]);
    const uint32_t off = info >> 16, deg = info & 0xFFFFu;
    for (uint32_t k = lane; k < deg; k += 64) {
        const uint32_t x = s_odst[off + k];
        atomicOr(&bm[x >> 5], 1u << (x & 31));
    }
}

// Relaxes the tile held in LDS rows D[v][64] to its local fixpoint.  On
// entry s_dirty marks the vertices whose rows were lowered from outside (and
// s_cand is clear); on exit s_dirty marks every row that changed.  Called by
// the whole workgroup.
template <int CAP, int NW>
__device__ __forceinline__ void relax_tile(uint32_t *D, const uint32_t *s_iinfo, const uint32_t *s_iarc,
                                           const uint32_t *s_oinfo, const uint16_t *s_odst,
                                           uint32_t (*s_cand)[CAP / 32], uint32_t *s_dirty,
                                           uint16_t *s_list, uint32_t *s_len, uint32_t wv, uint32_t lane) {
    constexpr uint32_t WORDS = CAP / 32;
    // first candidates: out-neighbours of every seeded vertex
    if (wv == 0) compact_bits<WORDS>(s_dirty, s_list, s_len, false);
    __syncthreads();
    {
        const uint32_t L = uniform(*s_len);
        for (uint32_t i = wv; i < L; i += NW) mark_out(s_cand[0], s_oinfo, s_odst, uniform(s_list[i]), lane);
    }
    __syncthreads();
    uint32_t cur = 0;
    for (;;) {
        if (wv == 0) compact_bits<WORDS>(s_cand[cur], s_list, s_len, true);
        __syncthreads();
        const uint32_t L = uniform(*s_len);
        if (L == 0) break;
        for (uint32_t i = wv; i < L; i += NW) {
            const uint32_t v = uniform(s_list[i]);
            if (pull_row<CAP>(D, s_iinfo, s_iarc, v, lane)) {
                if (lane == 0) atomicOr(&s_dirty[v >> 5], 1u << (v & 31));
                mark_out(s_cand[cur ^ 1u], s_oinfo, s_odst, v, lane);
            }
        }
        __syncthreads();
        cur ^= 1u;
    }
}

// Stages the in-tile in-arcs and out-arcs of tile [base, base+n) in LDS.
__device__ __forceinline__ void stage_tile_arcs(const SegPassArgs &A, uint32_t base, uint32_t n,
                                                uint32_t *s_iinfo, uint32_t *s_oinfo, uint32_t *s_iarc,
                                                uint16_t *s_odst) {
    const uint32_t ai = A.li_off[base], ao = A.l_off[base];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t i0 = A.li_off[base + i] - ai, i1 = A.li_off[base + i + 1] - ai;
        const uint32_t o0 = A.l_off[base + i] - ao, o1 = A.l_off[base + i + 1] - ao;
        s_iinfo[i] = (i0 << 16) | (i1 - i0);
        s_oinfo[i] = (o0 << 16) | (o1 - o0);
    }
    const uint32_t ni = A.li_off[base + n] - ai, no = A.l_off[base + n] - ao;
    for (uint32_t i = threadIdx.x; i < ni; i += blockDim.x) s_iarc[i] = A.li_arc[ai + i];
    for (uint32_t i = threadIdx.x; i < no; i += blockDim.x)
        s_odst[i] = static_cast<uint16_t>(A.l_arc[ao + i] >> 16);
}

// The same with the arcs reversed: a pull over out-arcs and marking over
// in-arcs, so relax_tile computes distances *to* the seeded vertices.
__device__ __forceinline__ void stage_tile_arcs_rev(const SegPassArgs &A, uint32_t base, uint32_t n,
                                                    uint32_t *s_iinfo, uint32_t *s_oinfo, uint32_t *s_iarc,
                                                    uint16_t *s_odst) {
    const uint32_t ai = A.l_off[base], ao = A.li_off[base];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t i0 = A.l_off[base + i] - ai, i1 = A.l_off[base + i + 1] - ai;
        const uint32_t o0 = A.li_off[base + i] - ao, o1 = A.li_off[base + i + 1] - ao;
        s_iinfo[i] = (i0 << 16) | (i1 - i0);
        s_oinfo[i] = (o0 << 16) | (o1 - o0);
    }
    const uint32_t ni = A.l_off[base + n] - ai, no = A.li_off[base + n] - ao;
    for (uint32_t i = threadIdx.x; i < ni; i += blockDim.x) s_iarc[i] = A.l_arc[ai + i];
    for (uint32_t i = threadIdx.x; i < no; i += blockDim.x)
        s_odst[i] = static_cast<uint16_t>(A.li_arc[ao + i] >> 16);
}

// Source-blocked pass: a workgroup relaxes one (tile, block of 64 sources)
// item at a time.  The tile's distances for the 64 sources sit in LDS as
// rows D[v][lane] (one 256-byte row per vertex); lanes are sources, so every
// LDS access of a wave is a whole row.  Relaxation is pull-based over a
// shared candidate bitmap: a candidate v takes, per lane, the minimum of
// D[v] and D[u] + w over its in-tile in-arcs; if any lane improved, v's
// in-tile out-neighbours become candidates of the next sweep and v is marked
// changed.  Each candidate is handled by one wave, so D[v] has one writer;
// reads of neighbours racing with their writers only see older upper
// bounds, which the candidate marking then revisits.  The boundary exchange
// and the activation of (block, tile) items are those of the one-source
// schedule, with inbox rows of 64 lanes.
template <int CAP, int NW>
__global__ __launch_bounds__(NW * 64) void k_segb_pass(SegPassArgs A) {
    constexpr uint32_t ACAP = 4u * CAP;
    constexpr uint32_t WORDS = CAP / 32;
    __shared__ uint32_t D[CAP * 64];
    __shared__ uint32_t s_iinfo[CAP];    // (in-arc offset << 16) | in-degree
    __shared__ uint32_t s_oinfo[CAP];    // (out-arc offset << 16) | out-degree
    __shared__ uint32_t s_iarc[ACAP];
    __shared__ uint16_t s_odst[ACAP];
    __shared__ uint32_t s_cand[2][WORDS];
    __shared__ uint32_t s_dirty[WORDS];
    __shared__ uint16_t s_list[CAP];
    __shared__ uint32_t s_len;
    __shared__ uint32_t s_unit;

    const uint32_t lane = lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    const uint32_t nunits = uniform(*A.nunits);
    const uint32_t stamp = uniform(*A.pass_ctr) + 1u;
    uint32_t staged = NONE;

    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(A.cursor, 1u);
        __syncthreads();
        const uint32_t u = uniform(s_unit);
        __syncthreads();
        if (u >= nunits) break;
        const uint2 unit = A.units[u];
        const uint32_t t = uniform(unit.x), slice = uniform(unit.y);
        const uint32_t base = uniform(A.tile_base[t]);
        const uint32_t n = uniform(A.tile_base[t + 1]) - base;
        if (t != staged) {
            stage_tile_arcs(A, base, n, s_iinfo, s_oinfo, s_iarc, s_odst);
            staged = t;
            __syncthreads();
        }
        const uint32_t total = uniform(A.cnt_cur[t]);
        const uint32_t first_k = slice * A.G;
        const uint32_t cnt = min(A.G, total - first_k);
        for (uint32_t k = 0; k < cnt; ++k) {
            const uint32_t b = uniform(A.bucket_cur[static_cast<size_t>(t) * A.S + first_k + k]);
            const size_t st = static_cast<size_t>(b) * A.T + t;
            const bool first = A.visited[st] == 0;
            uint32_t *gd = A.gdist + (static_cast<size_t>(b) * A.Vt + base) * 64;
            for (uint32_t v = wv; v < n; v += NW) D[v * 64 + lane] = first ? INF : gd[v * 64 + lane];
            for (uint32_t i = threadIdx.x; i < WORDS; i += blockDim.x) {
                s_cand[0][i] = 0;
                s_cand[1][i] = 0;
                s_dirty[i] = 0;
            }
            __syncthreads();
            // seeds: the block's own sources that lie in this tile
            if (wv == 0) {
                const uint32_t s = b * 64 + lane;
                if (s < A.nsrc && A.src_tile[s] == t) {
                    const uint32_t loc = A.src_pos[s] - base;
                    if (D[loc * 64 + lane] != 0) {
                        D[loc * 64 + lane] = 0;
                        atomicOr(&s_dirty[loc >> 5], 1u << (loc & 31));
                    }
                }
            }
            // seeds: inbox values that beat the stored ones
            const uint32_t p0 = uniform(A.port_base[t]), p1 = uniform(A.port_base[t + 1]);
            uint32_t *ib = A.inbox + static_cast<size_t>(b) * A.NP * 64;
            for (uint32_t kk = p0 + wv; kk < p1; kk += NW) {
                const uint32_t loc = uniform(A.port_local[kk]);
                const uint32_t v = ib[static_cast<size_t>(kk) * 64 + lane];
                const bool imp = v < D[loc * 64 + lane];
                if (imp) D[loc * 64 + lane] = v;
                if (__builtin_amdgcn_ballot_w64(imp) != 0 && lane == 0)
                    atomicOr(&s_dirty[loc >> 5], 1u << (loc & 31));
            }
            __syncthreads();
            relax_tile<CAP, NW>(D, s_iinfo, s_iarc, s_oinfo, s_odst, s_cand, s_dirty, s_list, &s_len, wv, lane);
            // write back: every row on the first visit, changed rows after
            for (uint32_t v = wv; v < n; v += NW)
                if (first || ((s_dirty[v >> 5] >> (v & 31)) & 1u)) gd[v * 64 + lane] = D[v * 64 + lane];
            if (threadIdx.x == 0 && first) A.visited[st] = 1;
            // boundary exchange of changed boundary-out vertices
            const uint32_t b0 = uniform(A.bo_base[t]), b1 = uniform(A.bo_base[t + 1]);
            for (uint32_t kk = b0 + wv; kk < b1; kk += NW) {
                const uint32_t loc = uniform(A.bo_local[kk]);
                if (!((s_dirty[loc >> 5] >> (loc & 31)) & 1u)) continue;
                const uint32_t dv = D[loc * 64 + lane];
                const uint32_t pos = base + loc;
                const uint32_t xe1 = uniform(A.x_off[pos + 1]);
                for (uint32_t xe = uniform(A.x_off[pos]); xe < xe1; ++xe) {
                    const uint32_t nd = sat_add(dv, uniform(A.x_w[xe]));
                    uint32_t *pi = ib + static_cast<size_t>(uniform(A.x_port[xe])) * 64 + lane;
                    const uint32_t t2 = uniform(A.x_tile[xe]);
                    bool imp = false;
                    if (nd < *pi) imp = nd < atomicMin(pi, nd);
                    if (__builtin_amdgcn_ballot_w64(imp) != 0 && lane == 0) seg_activate(A, b, t2, stamp);
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------- overlay schedule
// Boundary tables of one weight epoch, a workgroup per tile with lanes as
// seeds.  REV = false: F[pos][i] = in-tile distance from port i of the tile
// to pos (lanes = ports).  REV = true: B[pos][j] = in-tile distance from pos
// to exit j of the tile (lanes = exits, arcs reversed).  Lanes beyond the
// tile's ports / exits stay INF.
template <int CAP, int NW, bool REV>
__global__ __launch_bounds__(NW * 64) void k_ovl_custom(SegPassArgs A, uint32_t *__restrict__ F) {
    constexpr uint32_t ACAP = 4u * CAP;
    constexpr uint32_t WORDS = CAP / 32;
    __shared__ uint32_t D[CAP * 64];
    __shared__ uint32_t s_iinfo[CAP];
    __shared__ uint32_t s_oinfo[CAP];
    __shared__ uint32_t s_iarc[ACAP];
    __shared__ uint16_t s_odst[ACAP];
    __shared__ uint32_t s_cand[2][WORDS];
    __shared__ uint32_t s_dirty[WORDS];
    __shared__ uint16_t s_list[CAP];
    __shared__ uint32_t s_len;
    const uint32_t lane = lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    for (uint32_t t = blockIdx.x; t < A.T; t += gridDim.x) {
        const uint32_t base = uniform(A.tile_base[t]);
        const uint32_t n = uniform(A.tile_base[t + 1]) - base;
        if (REV)
            stage_tile_arcs_rev(A, base, n, s_iinfo, s_oinfo, s_iarc, s_odst);
        else
            stage_tile_arcs(A, base, n, s_iinfo, s_oinfo, s_iarc, s_odst);
        for (uint32_t v = wv; v < n; v += NW) D[v * 64 + lane] = INF;
        for (uint32_t i = threadIdx.x; i < WORDS; i += blockDim.x) {
            s_cand[0][i] = 0;
            s_cand[1][i] = 0;
            s_dirty[i] = 0;
        }
        __syncthreads();
        const uint32_t k0 = uniform(REV ? A.bo_base[t] : A.port_base[t]);
        const uint32_t k1 = uniform(REV ? A.bo_base[t + 1] : A.port_base[t + 1]);
        if (wv == 0 && lane < k1 - k0) {
            const uint32_t loc = REV ? A.bo_local[k0 + lane] : A.port_local[k0 + lane];
            D[loc * 64 + lane] = 0;
            atomicOr(&s_dirty[loc >> 5], 1u << (loc & 31));
        }
        __syncthreads();
        relax_tile<CAP, NW>(D, s_iinfo, s_iarc, s_oinfo, s_odst, s_cand, s_dirty, s_list, &s_len, wv, lane);
        uint32_t *Ft = F + static_cast<size_t>(base) * 64;
        for (uint32_t v = wv; v < n; v += NW) Ft[v * 64 + lane] = D[v * 64 + lane];
        __syncthreads();
    }
}

// First pass of the overlay schedule: a wave per source slot s (block
// s / 64, lane s % 64) sets the source's exit values to its in-tile distance
// to each exit j of its tile (lane j reads B[pos][j]) and flags the tiles the
// exit's cross arcs lead to.
__global__ void k_ovl_seed_push(SegPassArgs A, const uint32_t *__restrict__ B, const uint4 *__restrict__ hdr,
                                const uint32_t *__restrict__ bo_xbeg, const uint32_t *__restrict__ slots,
                                uint32_t nslots) {
    const uint32_t lane = lane_id();
    const uint32_t wpb = blockDim.x >> 6;
    for (uint32_t q = blockIdx.x * wpb + (threadIdx.x >> 6); q < nslots; q += gridDim.x * wpb) {
        const uint32_t s = uniform(slots ? slots[q] : q);
        const uint32_t t = uniform(A.src_tile[s]);
        if (t == NONE) continue;
        const uint32_t b = s >> 6, l = s & 63u;
        const uint32_t pos = uniform(A.src_pos[s]);
        const uint4 h = hdr[t];
        const uint32_t b0 = uniform(h.y), xa0 = uniform(h.z), X = (uniform(h.w) >> 8) & 0xFFu;
        if (lane >= X) continue;
        const uint32_t d = B[static_cast<size_t>(pos) * 64 + lane];
        if (d == INF) continue;
        A.xval[(static_cast<size_t>(b) * A.NB + b0 + lane) * 64 + l] = d;
        const uint32_t k1 = bo_xbeg[b0 + t + lane + 1];
        for (uint32_t k = bo_xbeg[b0 + t + lane]; k < k1; ++k)
            A.flags[static_cast<size_t>(A.x_tile[xa0 + k]) * A.S + b] = 1;
    }
}

// In-tile distances for sources that share a tile with some target: a
// workgroup per group of up to 64 sources in one tile (lanes = sources)
// relaxes the tile from them in LDS and lowers out[...] to the in-tile value
// (paths that leave the tile are in out[...] already).  pairs mode: the
// group's entries (lane << 16 | target local index, output index);
// full mode (pairs == NULL): every vertex of the tile for every lane, at
// out[row[lane] * V + vertex].  With pair_val, pairs mode stores the in-tile
// values there instead (k_min_scatter applies them later).
struct IntileGroup {
    uint32_t tile, lanes, p0, p1;
};
template <int CAP, int NW>
__global__ __launch_bounds__(NW * 64) void k_intile_fix(SegPassArgs A, const IntileGroup *__restrict__ groups,
                                                         uint32_t ngroups, const uint32_t *__restrict__ src_local,
                                                         const uint32_t *__restrict__ pair_key,
                                                         const uint64_t *__restrict__ pair_out,
                                                         const uint32_t *__restrict__ row,
                                                         const uint32_t *__restrict__ vert_of, uint32_t V,
                                                         uint32_t *__restrict__ out, uint32_t *__restrict__ pair_val) {
    constexpr uint32_t ACAP = 4u * CAP;
    constexpr uint32_t WORDS = CAP / 32;
    __shared__ uint32_t D[CAP * 64];
    __shared__ uint32_t s_iinfo[CAP];
    __shared__ uint32_t s_oinfo[CAP];
    __shared__ uint32_t s_iarc[ACAP];
    __shared__ uint16_t s_odst[ACAP];
    __shared__ uint32_t s_cand[2][WORDS];
    __shared__ uint32_t s_dirty[WORDS];
    __shared__ uint16_t s_list[CAP];
    __shared__ uint32_t s_len;
    const uint32_t lane = lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    for (uint32_t gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
        const IntileGroup G = groups[gi];
        const uint32_t t = uniform(G.tile), nl = uniform(G.lanes);
        const uint32_t base = uniform(A.tile_base[t]);
        const uint32_t n = uniform(A.tile_base[t + 1]) - base;
        stage_tile_arcs(A, base, n, s_iinfo, s_oinfo, s_iarc, s_odst);
        for (uint32_t v = wv; v < n; v += NW) D[v * 64 + lane] = INF;
        for (uint32_t i = threadIdx.x; i < WORDS; i += blockDim.x) {
            s_cand[0][i] = 0;
            s_cand[1][i] = 0;
            s_dirty[i] = 0;
        }
        __syncthreads();
        if (wv == 0 && lane < nl) {
            const uint32_t loc = src_local[static_cast<size_t>(gi) * 64 + lane];
            D[loc * 64 + lane] = 0;
            atomicOr(&s_dirty[loc >> 5], 1u << (loc & 31));
        }
        __syncthreads();
        relax_tile<CAP, NW>(D, s_iinfo, s_iarc, s_oinfo, s_odst, s_cand, s_dirty, s_list, &s_len, wv, lane);
        if (pair_key) {
            for (uint32_t q = G.p0 + threadIdx.x; q < G.p1; q += blockDim.x) {
                const uint32_t key = pair_key[q];
                const uint32_t d = D[(key & 0xFFFFu) * 64 + (key >> 16)];
                if (pair_val) {
                    pair_val[q] = d;
                } else {
                    uint32_t *o = out + pair_out[q];
                    *o = min(*o, d);
                }
            }
        } else if (lane < nl) {
            const uint64_t r = static_cast<uint64_t>(row[static_cast<size_t>(gi) * 64 + lane]) * V;
            for (uint32_t v = wv; v < n; v += NW) {
                uint32_t *o = out + r + vert_of[base + v];
                *o = min(*o, D[v * 64 + lane]);
            }
        }
        __syncthreads();
    }
}

// out[idx[q]] = min(out[idx[q]], val[q]) for every q < n.
__global__ void k_min_scatter(const uint64_t *__restrict__ idx, const uint32_t *__restrict__ val, uint32_t n,
                              uint32_t *__restrict__ out) {
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
        out[idx[q]] = min(out[idx[q]], val[q]);
}

// Overlay pass: a visit of (tile t, block b) computes the block's value at
// the head of every cross arc a = (e -> p) into t from the exit values of
// the neighbouring tiles (entry_a = xval[e] + w_a), maps them through t's
// table onto t's exits (exit_j = min_a entry_a + F[exit_j][p(a)], a dense
// min-plus product, which also takes the minimum over the arcs of a port),
// and stores each exit value that dropped, flagging the tiles that exit's
// cross arcs lead to for the next pass.  All traffic is
// plain loads and stores: a pass reads the exit values the previous passes
// wrote (kernel boundaries order them), and a flag set during a pass brings
// its tile back in the next one.
//
// A workgroup takes one unit (a tile and up to G of its active blocks),
// stages the tile's packed table rows (one column per incoming cross arc),
// its incoming arcs and its exits' outgoing arcs in LDS, and runs the unit's
// visits one after another.  Wave w owns entry rows w, w + NW, ... (R of
// them; row i is incoming arc i, whose source exit and weight are the same
// for the whole wave) and exits w R .. w R + R - 1: per visit it loads its
// entry rows, the current values of its exits and its bound with all loads
// in flight.  Visits are software-pipelined two deep: once a visit's entry
// rows are in LDS its registers take the loads of the visit two ahead, so
// every visit's rows have two visits' time to arrive.  Rows and exits past
// the tile's last are clamped to it (loaded again, never stored), so every
// load is unconditional.  LDS is sized at launch to the tiling's largest
// tile (XM exits x EM entries, PM arcs in or out); R is the smallest
// instance with NW R >= max(EM, XM).
constexpr uint32_t OVL_XCAP = 64;     // exits per tile (one 64-lane row of the exit table)
constexpr uint32_t OVL_ECAP = 64;     // incoming cross arcs per tile (table columns)
constexpr uint32_t OVL_PCAP = 512;    // cross arcs leaving a tile
constexpr uint32_t OVL_NW = 8;        // waves per workgroup
constexpr uint64_t OVL_UNIT_PERM = 2654435761ull;   // a prime above any unit count (see seg_units_cap)
template <int NW, int R>
__global__ __launch_bounds__(NW * 64, R <= 4 ? 8 : 1) void k_ovl_pass(SegPassArgs A, const uint32_t *__restrict__ Fx,
                                                                     const uint4 *__restrict__ hdr,
                                                                     const uint32_t *__restrict__ bo_xbeg, uint32_t XM,
                                                                     uint32_t EM, uint32_t PM) {
    HIP_DYNAMIC_SHARED(uint32_t, lds)
    uint32_t *s_M = lds;                     // [XM][EM]     table rows of the exits
    uint32_t *s_in0 = s_M + XM * EM;         // [2][EM][64]  entry values, by visit parity
    uint32_t *s_xbeg = s_in0 + 2 * EM * 64;  // [XM + 1]     first outgoing arc of each exit
    uint32_t *s_xtile = s_xbeg + XM + 1;     // [PM]         outgoing arcs: target tile
    uint32_t *s_pexit = s_xtile + PM;        // [PM]         incoming arcs: source exit,
    uint32_t *s_pw = s_pexit + PM;           //              weight
    uint32_t *s_unit = s_pw + PM;
    const uint32_t lane = lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    const uint32_t nunits = uniform(*A.nunits);
    static_assert(NW * 64 >= OVL_PCAP && NW * 64 >= OVL_ECAP, "one staging round covers a tile's arcs");
    // Workgroup w takes unit w first, then units gridDim + cursor++ until
    // the end, so each unit is taken once; workgroups with no first unit
    // leave at once (light passes), and none waits on the cursor to start.
    uint32_t u = blockIdx.x;
    if (u >= nunits) return;
    uint32_t staged = NONE;
    uint32_t stored = 0;   // exit values this wave stored (uniform)
    for (;;) {
        // units are taken in a scattered order (u -> u * P mod nunits, a
        // bijection for the prime P > nunits): each pass then moves every
        // front about one tile instead of cascading along the tiles' order,
        // which lowers the visits to convergence
        const uint2 unit = A.units[static_cast<uint32_t>((static_cast<uint64_t>(u) * OVL_UNIT_PERM) % nunits)];
        const uint32_t t = uniform(unit.x), slice = uniform(unit.y);
        // every load that depends on the tile alone is issued before any of
        // them is used (one round trip): its header, its incoming-arc range,
        // its active count and the unit's block ids (one per lane, clamped
        // into the tile's row; only lanes below the unit's count are used)
        const uint4 h = hdr[t];
        const uint2 h2 = A.hdr2[t];
        const uint32_t tot = A.cnt_cur[t];
        const uint32_t first_k = slice * A.G;
        const uint32_t blk = A.bucket_cur[static_cast<size_t>(t) * A.S + min(first_k + lane, A.S - 1)];
        const uint32_t b0 = uniform(h.y), xa0 = uniform(h.z), hw = uniform(h.w);
        const uint32_t X = (hw >> 8) & 0xFFu, na = hw >> 16;
        const uint32_t total = uniform(tot), pa0 = uniform(h2.x), npa = uniform(h2.y);
        const bool work = npa != 0 && X != 0;
        if (work && t != staged) {
            // staging, again in one round: thread q loads entry q of every
            // staged array before writing any (a tile with exits has at
            // least one arc leaving it, so the clamped indices stay in its
            // ranges); only table rows can outnumber the threads
            const uint32_t q = threadIdx.x;
            const uint32_t *rows = Fx + static_cast<size_t>(b0) * EM;
            const uint32_t nM = X * EM;
            const uint32_t vM = rows[min(q, nM - 1)];
            const uint32_t vX = bo_xbeg[b0 + t + min(q, X)];
            const uint32_t vT = A.x_tile[xa0 + min(q, na - 1)];
            const uint2 vR = A.pin_rec[pa0 + min(q, npa - 1)];
            if (q < nM) s_M[q] = vM;
            if (q <= X) s_xbeg[q] = vX;
            if (q < na) s_xtile[q] = vT;
            if (q < npa) {
                s_pexit[q] = vR.x;
                s_pw[q] = vR.y & 0xFFFFu;
            }
#pragma unroll 4
            for (uint32_t i = q + blockDim.x; i < nM; i += blockDim.x) s_M[i] = rows[i];
            staged = t;
            __syncthreads();
        }
        const uint32_t cnt = work ? min(A.G, total - first_k) : 0u;
        if (cnt != 0) {
            const uint32_t elast = npa - 1, xlast = X - 1;
            // per entry row of this wave: its arc's source exit and weight
            // (uniform, and the same for every visit of the unit)
            uint32_t erow[R], ew[R];
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) {
                const uint32_t k0 = min(wv + NW * r, elast);
                erow[r] = uniform(s_pexit[k0]);
                ew[r] = uniform(s_pw[k0]);
            }
            // a visit's loads into one register set: its entry rows, its
            // exits' current values and its target bound (without bounds a
            // row of the block is read instead, through a select rather than
            // a branch, so every load is unconditional and the waits on them
            // stay exact)
            auto issue = [&](uint32_t (&vn)[R], uint32_t (&cn)[R], uint32_t &bn, uint32_t bid) {
                const uint32_t *xb = A.xval + static_cast<size_t>(bid) * A.NB * 64;
                const uint32_t *xv = xb + static_cast<size_t>(b0) * 64;
                const uint32_t *bp = A.bound ? A.bound + static_cast<size_t>(bid) * 64 : xb;
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) vn[r] = xb[static_cast<size_t>(erow[r]) * 64 + lane];
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) cn[r] = xv[static_cast<size_t>(min(wv * R + r, xlast)) * 64 + lane];
                bn = bp[lane];
            };
            auto visit = [&](uint32_t k, uint32_t (&vn)[R], uint32_t (&cn)[R], uint32_t &bn) {
                const uint32_t b = __builtin_amdgcn_readlane(blk, k);
                // target-bounded passes: a value above the lane's bound is
                // never on a shortest path to one of its source's targets
                const uint32_t bnd = A.bound ? bn : INF;
                uint32_t *xv = A.xval + (static_cast<size_t>(b) * A.NB + b0) * 64;  // own exit j at xv + 64 j
                // entry rows alternate between two buffers: a wave that
                // starts the next visit writes the other one while slower
                // waves may still read this one, and the visit after that
                // writes here only once every wave has passed the next
                // visit's barrier
                uint32_t *s_in = s_in0 + (k & 1u) * EM * 64;
                uint32_t c[R];
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) c[r] = cn[r];
#pragma unroll
                for (uint32_t r = 0; r < R; ++r) {
                    const uint32_t i = wv + NW * r;
                    if (i < npa) s_in[i * 64 + lane] = sat_add(vn[r], ew[r]);
                }
                // this register set now takes the loads of the visit two
                // ahead; they go out before the barrier, so that the wait
                // there and this visit's exits overlap them.  Past the unit's
                // last visit this block's rows are loaded again (cache hits):
                // issuing always keeps each set in its registers across the
                // loop, where a conditional issue would make the compiler
                // copy registers whose loads are still in flight
                issue(vn, cn, bn, k + 2 < cnt ? __builtin_amdgcn_readlane(blk, min(k + 2, 63u)) : b);
                __syncthreads();
                // this wave's exits (rows past the tile's last repeat it):
                // min-plus over the entry rows; rows past the tile's arcs
                // are not written this visit, their table entries are INF
                // and a saturating add with INF is INF whatever the row holds
                const uint32_t j0 = wv * R;
                if (j0 < X) {
                    uint32_t m[R];
#pragma unroll
                    for (uint32_t r = 0; r < R; ++r) m[r] = INF;
                    for (uint32_t i = 0; i < npa; i += 4) {
                        const uint32_t e0 = s_in[i * 64 + lane], e1 = s_in[(i + 1) * 64 + lane];
                        const uint32_t e2 = s_in[(i + 2) * 64 + lane], e3 = s_in[(i + 3) * 64 + lane];
#pragma unroll
                        for (uint32_t r = 0; r < R; ++r) {
                            const uint4 f = *reinterpret_cast<const uint4 *>(s_M + min(j0 + r, xlast) * EM + i);
                            m[r] = min(m[r], min(min(sat_add(e0, f.x), sat_add(e1, f.y)),
                                                 min(sat_add(e2, f.z), sat_add(e3, f.w))));
                        }
                    }
                    // exits that dropped: store the value, flag the arcs' targets
#pragma unroll
                    for (uint32_t r = 0; r < R; ++r) {
                        const uint32_t j = j0 + r;
                        if (j >= X) break;
                        const bool imp = m[r] < c[r] && m[r] <= bnd;
                        if (imp) xv[static_cast<size_t>(j) * 64 + lane] = m[r];
                        const uint64_t bal = __builtin_amdgcn_ballot_w64(imp);
                        stored += static_cast<uint32_t>(__builtin_popcountll(bal));
                        if (bal == 0) continue;
                        const uint32_t kb = uniform(s_xbeg[j]), ke = uniform(s_xbeg[j + 1]);
                        for (uint32_t kx = kb + lane; kx < ke; kx += 64)
                            A.flags[static_cast<size_t>(s_xtile[kx]) * A.S + b] = 1;
                    }
                }
            };
            uint32_t vn0[R], cn0[R], bn0, vn1[R], cn1[R], bn1;
            const uint32_t blk0 = __builtin_amdgcn_readfirstlane(blk);
            issue(vn0, cn0, bn0, blk0);
            issue(vn1, cn1, bn1, cnt > 1 ? __builtin_amdgcn_readlane(blk, 1) : blk0);
            uint32_t k = 0;
            for (; k + 1 < cnt; k += 2) {
                visit(k, vn0, cn0, bn0);
                visit(k + 1, vn1, cn1, bn1);
            }
            if (k < cnt) visit(k, vn0, cn0, bn0);
        }
        // the unit's last visit ends without a barrier: every wave passes
        // the two below before the next unit stages or writes entry rows
        if (threadIdx.x == 0) *s_unit = gridDim.x + atomicAdd(A.cursor, 1u);
        __syncthreads();
        u = uniform(*s_unit);
        __syncthreads();
        if (u >= nunits) break;
    }
    if (lane == 0 && stored) A.wave_stores[blockIdx.x * NW + wv] += stored;
}

// Builds the pass's work lists from the activation flags [tile][block]:
// each tile's active blocks in ascending order, the tile's count, and units
// of G blocks counted in *nunits (zeroed by the previous pass's plan); clears
// the flags it consumed, counts visits per tile, and zeroes the next pass's
// unit count, unit cursor and pending-work counters (total and per block).
// A wave scans one tile; the waves of a workgroup reserve their units with
// one atomic between them (OVL_PLAN_WAVES waves per workgroup).
constexpr uint32_t OVL_PLAN_WAVES = 16;
__global__ __launch_bounds__(OVL_PLAN_WAVES * 64) void k_ovl_plan(
    uint8_t *__restrict__ flags, uint32_t T, uint32_t S, uint32_t *__restrict__ cnt, uint32_t *__restrict__ bucket,
    uint32_t G, uint2 *__restrict__ units, uint32_t *__restrict__ nunits, uint32_t *__restrict__ next_nunits,
    uint32_t *__restrict__ next_cursor, uint32_t *__restrict__ next_pending, uint32_t *__restrict__ row_pending,
    unsigned long long *__restrict__ stats, uint32_t *__restrict__ tile_visits) {
    __shared__ uint32_t s_off[OVL_PLAN_WAVES];
    __shared__ uint32_t s_base;
    const uint32_t lane = lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *next_nunits = 0;
        *next_cursor = 0;
        *next_pending = 0;
    }
    if (blockIdx.x == 0)
        for (uint32_t b = threadIdx.x; b < S; b += blockDim.x) row_pending[b] = 0;
    // every wave of the workgroup runs the same iterations (the barriers)
    for (uint32_t t0 = blockIdx.x * OVL_PLAN_WAVES; t0 < T; t0 += gridDim.x * OVL_PLAN_WAVES) {
        const uint32_t t = t0 + wv;
        uint32_t k = 0;
        if (t < T) {
            uint8_t *f = flags + static_cast<size_t>(t) * S;
            uint32_t *bk = bucket + static_cast<size_t>(t) * S;
            // the row's flags 512 at a time: all eight loads of a lane are
            // issued before the first ballot (indices clamped into the row),
            // so a row costs one round trip, not one per 64 blocks
            for (uint32_t g0 = 0; g0 < S; g0 += 512) {
                uint32_t v[8];
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) v[q] = f[min(g0 + q * 64 + lane, S - 1)];
#pragma unroll
                for (uint32_t q = 0; q < 8; ++q) {
                    const uint32_t b = g0 + q * 64 + lane;
                    const bool on = b < S && v[q] != 0;
                    const uint64_t msk = __builtin_amdgcn_ballot_w64(on);
                    if (on) {
                        bk[k + mbcnt64(msk)] = b;
                        f[b] = 0;
                    }
                    k += static_cast<uint32_t>(__builtin_popcountll(msk));
                }
            }
            if (lane == 0) {
                cnt[t] = k;
                if (k) tile_visits[t] += k;   // this wave owns tile t in this pass
            }
        }
        const uint32_t sl = (k + G - 1) / G;
        if (lane == 0) s_off[wv] = sl;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
            for (uint32_t i = 0; i < OVL_PLAN_WAVES; ++i) {
                const uint32_t x = s_off[i];
                s_off[i] = tot;
                tot += x;
            }
            uint32_t base = 0;
            if (tot) {
                base = atomicAdd(nunits, tot);
                if (base == 0) atomicAdd(&stats[1], 1ull);
            }
            s_base = base;
        }
        __syncthreads();
        const uint32_t ub = s_base + s_off[wv];
        for (uint32_t q = lane; q < sl; q += 64) units[ub + q] = make_uint2(t, q);
        __syncthreads();   // s_off and s_base are rewritten by the next iteration
    }
}

// Packs the exits' rows of the boundary tables with one column per incoming
// cross arc of the tile (arcs in the order of their records, grouped by
// port): Fx[exit][i] = F[pos][port of arc i], INF for i up to the row length
// EM.  A port reached by several arcs repeats its column, so a pass takes
// the minimum over those arcs in its min-plus step.
__global__ void k_ovl_pack(const uint32_t *__restrict__ F, const uint32_t *__restrict__ tile_base,
                           const uint32_t *__restrict__ bo_local, const uint4 *__restrict__ hdr,
                           const uint2 *__restrict__ hdr2, const uint32_t *__restrict__ pin_lport, uint32_t T,
                           uint32_t EM, uint32_t *__restrict__ Fx) {
    const uint32_t lane = lane_id();
    const uint32_t wpb = blockDim.x >> 6;
    for (uint32_t t = blockIdx.x * wpb + (threadIdx.x >> 6); t < T; t += gridDim.x * wpb) {
        const uint32_t base = tile_base[t];
        const uint4 h = hdr[t];
        const uint2 h2 = hdr2[t];
        const uint32_t b0 = h.y, X = (h.w >> 8) & 0xFFu, pa0 = h2.x, npa = h2.y;
        for (uint32_t j = 0; j < X; ++j) {
            const uint32_t pos = base + bo_local[b0 + j];
            for (uint32_t i = lane; i < EM; i += 64)
                Fx[static_cast<size_t>(b0 + j) * EM + i] =
                    i < npa ? F[static_cast<size_t>(pos) * 64 + pin_lport[pa0 + i]] : INF;
        }
    }
}

// Adds 1 to *out for every wave that sees a set flag (pending work) and
// marks row_pending[b] for every block b with a set flag (flags are [T][S]).
__global__ void k_flags_any(const uint8_t *__restrict__ flags, size_t n, uint32_t S, uint32_t *__restrict__ out,
                            uint32_t *__restrict__ row_pending) {
    bool any = false;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        if (flags[i] != 0) {
            any = true;
            row_pending[i % S] = 1;
        }
    }
    if (__builtin_amdgcn_ballot_w64(any) != 0 && lane_id() == 0) atomicAdd(out, 1u);
}

// Distance of chunk source s (vertex src_v) to v under the overlay schedule
// over paths that leave the source's tile: the minimum, over the cross arcs
// e -> p into v's tile, of the arc's source exit value xval[e] + w + F[v][p]
// (the per-port minimum of the pass, folded into one loop over the tile's
// contiguous arc records).  The source itself is 0; paths that stay inside
// the source's tile are added by k_intile_fix.
struct OvlRead {
    const uint32_t *tile_of, *pos_of, *xval, *F;
    const uint2 *hdr2, *pin_rec;
    uint32_t NB;
};
__device__ __forceinline__ uint32_t ovl_value(const OvlRead &R, uint32_t s, uint32_t src_v, uint32_t v) {
    if (v == src_v) return 0u;
    const uint32_t t = R.tile_of[v];
    if (t == NONE) return INF;
    const size_t b = s >> 6, l = s & 63u;
    const uint32_t pos = R.pos_of[v];
    const uint2 h2 = R.hdr2[t];
    const uint2 *rec = R.pin_rec + h2.x;
    const uint32_t *xb = R.xval + (b * R.NB) * 64 + l;
    const uint32_t *Fv = R.F + static_cast<size_t>(pos) * 64;
    uint32_t m = INF;
#pragma unroll 4
    for (uint32_t k = 0; k < h2.y; ++k) {
        const uint2 r = rec[k];
        m = min(m, sat_add(sat_add(xb[static_cast<size_t>(r.x) * 64], r.y & 0xFFFFu), Fv[r.y >> 16]));
    }
    return m;
}

// Full distance rows under the overlay schedule, one workgroup per (tile,
// row group) item; a row group is a block of 64 chunk sources with the
// output row of each lane (NONE where that source's row is not wanted).
// The block's entry values at the tile's ports are pulled once into LDS
// (min over the tile's incoming cross arcs of exit value + w), then every
// vertex of the tile takes min over the ports of entry + F[vertex][port]
// (its table row, one coalesced load, broadcast port by port).  A wave
// computes 32 vertices for its 64 sources into LDS and stores them
// transposed, two rows per instruction over consecutive tile positions.
// Rows are INF-filled before and their sources set to 0 after (k_fill_rows,
// k_rows_src_zero); paths inside a source's own tile come from the in-tile
// fix-up.
constexpr uint32_t ROWS_NW = 4;      // waves per workgroup
constexpr uint32_t ROWS_CHUNK = 32;  // vertices a wave stages at a time
__global__ __launch_bounds__(ROWS_NW * 64) void k_ovl_rows(OvlRead R, const uint32_t *__restrict__ tile_base,
                                                           const uint4 *__restrict__ hdr, uint32_t T,
                                                           const uint32_t *__restrict__ grp_block,
                                                           const uint32_t *__restrict__ lane_row, uint64_t items,
                                                           const uint32_t *__restrict__ vert_of, uint32_t V,
                                                           uint32_t *__restrict__ out) {
    HIP_DYNAMIC_SHARED(uint32_t, lds)
    uint32_t *s_row = lds;                        // [64] output row of each source lane
    uint32_t *s_val = s_row + 64;                 // [ROWS_NW][ROWS_CHUNK][65] staged values
    uint32_t *s_ent = s_val + ROWS_NW * ROWS_CHUNK * 65;   // [most ports of a tile][64]
    const uint32_t lane = lane_id();
    const uint32_t wv = uniform(threadIdx.x >> 6);
    uint32_t *sv = s_val + wv * ROWS_CHUNK * 65;
    const uint32_t j = lane & (ROWS_CHUNK - 1), h = lane / ROWS_CHUNK;   // store phase: vertex, row parity
    for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const uint32_t t = uniform(static_cast<uint32_t>(it % T)), gi = uniform(static_cast<uint32_t>(it / T));
        const uint32_t b = uniform(grp_block[gi]);
        const uint32_t E = uniform(hdr[t].w & 0xFFu);
        const uint2 h2 = R.hdr2[t];
        const uint32_t a0 = uniform(h2.x), na = uniform(h2.y);
        const uint32_t base = uniform(tile_base[t]), n = uniform(tile_base[t + 1]) - base;
        if (threadIdx.x < 64) s_row[lane] = lane_row[static_cast<size_t>(gi) * 64 + lane];
        for (uint32_t i = wv; i < E; i += ROWS_NW) s_ent[i * 64 + lane] = INF;
        __syncthreads();
        const uint32_t *xb = R.xval + static_cast<size_t>(b) * R.NB * 64 + lane;
        for (uint32_t k = wv; k < na; k += ROWS_NW) {
            const uint2 rec = R.pin_rec[a0 + k];
            atomicMin(&s_ent[(rec.y >> 16) * 64 + lane], sat_add(xb[static_cast<size_t>(rec.x) * 64], rec.y & 0xFFFFu));
        }
        __syncthreads();
        for (uint32_t c0 = wv * ROWS_CHUNK; c0 < n; c0 += ROWS_NW * ROWS_CHUNK) {
            const uint32_t cn = min(ROWS_CHUNK, n - c0);
            for (uint32_t q = 0; q < cn; ++q) {
                const uint32_t fv = R.F[static_cast<size_t>(base + c0 + q) * 64 + lane];
                uint32_t m = INF;
                for (uint32_t i = 0; i < E; ++i)
                    m = min(m, sat_add(s_ent[i * 64 + lane], __builtin_amdgcn_readlane(fv, i)));
                sv[q * 65 + lane] = m;
            }
            __builtin_amdgcn_wave_barrier();
            const uint32_t vj = j < cn ? vert_of[base + c0 + j] : 0u;
            for (uint32_t l2 = 0; l2 < 32; ++l2) {
                const uint32_t l = 2 * l2 + h;
                const uint32_t r = s_row[l];
                if (j < cn && r != NONE) out[static_cast<size_t>(r) * V + vj] = sv[j * 65 + l];
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

// out[out_row[r] * V + v] = value for every v < V of each listed row.
__global__ void k_fill_rows(uint32_t *__restrict__ out, uint32_t V, uint32_t rows,
                            const uint32_t *__restrict__ out_row, uint32_t value) {
    for (uint32_t r = blockIdx.y; r < rows; r += gridDim.y) {
        uint32_t *o = out + static_cast<size_t>(out_row[r]) * V;
        for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) o[v] = value;
    }
}

// Each row's source is at distance 0 from itself.
__global__ void k_rows_src_zero(uint32_t *__restrict__ out, uint32_t V, uint32_t rows,
                                const uint32_t *__restrict__ out_row, const uint32_t *__restrict__ row_vertex) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
        out[static_cast<size_t>(out_row[r]) * V + row_vertex[r]] = 0;
}

// One order per blockIdx.x (strided), its P x P pairs spread over the
// threads of gridDim.y workgroups.
__global__ void k_gather_ovl(uint32_t num_orders, const uint32_t *__restrict__ pick_off,
                             const uint32_t *__restrict__ picks, const uint64_t *__restrict__ out_base,
                             const uint32_t *__restrict__ src_idx_of_pick, uint32_t lo, uint32_t n, OvlRead R,
                             uint32_t *__restrict__ out) {
    for (uint32_t o = blockIdx.x; o < num_orders; o += gridDim.x) {
        const uint32_t a = pick_off[o], P = pick_off[o + 1] - a;
        const uint64_t ob = out_base[o];
        for (uint32_t k = blockIdx.y * blockDim.x + threadIdx.x; k < P * P; k += gridDim.y * blockDim.x) {
            const uint32_t i = k / P, j = k - i * P;
            const uint32_t si = src_idx_of_pick[a + i];
            if (si < lo || si >= lo + n) continue;
            out[ob + k] = ovl_value(R, si - lo, picks[a + i], picks[a + j]);
        }
    }
}

// Target bounds: tmp[s] = max over the (i, j) pairs of the orders whose
// source pick i is chunk source s of the current overlay value d(s, p_j),
// the length of a path already found (INF while some target is unreached);
// tmp must be 0 before.  k_bound_min then keeps the smaller of the old
// bound and tmp.
__global__ void k_bound_pairs(uint32_t num_orders, const uint32_t *__restrict__ pick_off,
                              const uint32_t *__restrict__ picks, const uint32_t *__restrict__ src_idx_of_pick,
                              uint32_t lo, uint32_t n, OvlRead R, uint32_t *__restrict__ tmp) {
    for (uint32_t o = blockIdx.x; o < num_orders; o += gridDim.x) {
        const uint32_t a = pick_off[o], P = pick_off[o + 1] - a;
        for (uint32_t k = blockIdx.y * blockDim.x + threadIdx.x; k < P * P; k += gridDim.y * blockDim.x) {
            const uint32_t i = k / P, j = k - i * P;
            const uint32_t si = src_idx_of_pick[a + i];
            if (si < lo || si >= lo + n) continue;
            atomicMax(&tmp[si - lo], ovl_value(R, si - lo, picks[a + i], picks[a + j]));
        }
    }
}

__global__ void k_bound_min(uint32_t *__restrict__ bound, uint32_t *__restrict__ tmp, uint32_t n) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        bound[s] = min(bound[s], tmp[s]);
        tmp[s] = 0;
    }
}

// Seeds pass 0: (s, tile of source s) for every source with a tile.
__global__ void k_seg_seed(SegPassArgs A, uint32_t n, uint32_t lanes_log2) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t t = A.src_tile[s];
    if (t != NONE) seg_activate(A, s >> lanes_log2, t, 1u);
}

// Splits every active tile's bucket into units of G sources, zeroes the
// unit cursor and the next-pass counters, and counts work.
__global__ void k_seg_plan(const uint32_t *__restrict__ tiles_cur,
                           const uint32_t *__restrict__ ntiles_cur,
                           const uint32_t *__restrict__ cnt_cur, uint32_t G,
                           uint2 *__restrict__ units, uint32_t *__restrict__ nunits,
                           unsigned long long *__restrict__ stats) {
    const uint32_t nt = *ntiles_cur;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < nt; j += gridDim.x * blockDim.x) {
        const uint32_t t = tiles_cur[j];
        const uint32_t c = cnt_cur[t];
        const uint32_t sl = (c + G - 1) / G;
        const uint32_t b = atomicAdd(nunits, sl);
        for (uint32_t k = 0; k < sl; ++k) units[b + k] = make_uint2(t, k);
        atomicAdd(&stats[0], static_cast<unsigned long long>(c));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && nt) atomicAdd(&stats[1], 1ull);
}

// Zeroes the next pass's activation counters; bumps the pass counter.
__global__ void k_seg_prologue(uint32_t *__restrict__ cnt_next, uint32_t T,
                               uint32_t *__restrict__ ntiles_next, uint32_t *__restrict__ nunits,
                               uint32_t *__restrict__ cursor, uint32_t *__restrict__ pass_ctr) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x)
        cnt_next[t] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *ntiles_next = 0;
        *nunits = 0;
        *cursor = 0;
        *pass_ctr += 1u;
    }
}

// Final distance of chunk source s at vertex v from the segmented state
// (lanes_log2 = 0: one source per state row; 6: blocks of 64 sources).
__device__ __forceinline__ uint32_t seg_value(const uint32_t *tile_of, const uint32_t *pos_of,
                                              const uint8_t *visited, const uint32_t *gdist,
                                              uint32_t T, uint32_t Vt, uint32_t lanes_log2,
                                              uint32_t s, uint32_t src_v, uint32_t v) {
    const uint32_t t = tile_of[v];
    if (t == NONE) return v == src_v ? 0u : INF;
    const size_t b = s >> lanes_log2, l = s & ((1u << lanes_log2) - 1u);
    if (!visited[b * T + t]) return INF;
    return gdist[((b * Vt + pos_of[v]) << lanes_log2) + l];
}

__global__ void k_seg_emit(const uint32_t *__restrict__ tile_of, const uint32_t *__restrict__ pos_of,
                           const uint8_t *__restrict__ visited, const uint32_t *__restrict__ gdist,
                           uint32_t T, uint32_t Vt, uint32_t lanes_log2, uint32_t V, uint32_t rows,
                           const uint32_t *__restrict__ row_src_idx,
                           const uint32_t *__restrict__ row_src_vertex,
                           const uint32_t *__restrict__ out_row, uint32_t *__restrict__ out) {
    for (uint32_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const uint32_t s = row_src_idx[r], sv = row_src_vertex[r];
        uint32_t *o = out + static_cast<size_t>(out_row[r]) * V;
        for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x)
            o[v] = seg_value(tile_of, pos_of, visited, gdist, T, Vt, lanes_log2, s, sv, v);
    }
}


// ---------------------------------------------------------- order gathers
// One workgroup per order; entry (i, j) of order o is written at
// out_base[o] + i*P + j.
__global__ void k_gather_rows(uint32_t num_orders, const uint32_t *__restrict__ pick_off,
                              const uint32_t *__restrict__ picks,
                              const uint64_t *__restrict__ out_base,
                              const uint32_t *__restrict__ row_of_pick,
                              const uint32_t *__restrict__ rows, uint32_t V,
                              uint32_t *__restrict__ out) {
    for (uint32_t o = blockIdx.x; o < num_orders; o += gridDim.x) {
        const uint32_t a = pick_off[o], P = pick_off[o + 1] - a;
        const uint64_t ob = out_base[o];
        for (uint32_t k = threadIdx.x; k < P * P; k += blockDim.x) {
            const uint32_t i = k / P, j = k - i * P;
            out[ob + k] = rows[static_cast<size_t>(row_of_pick[a + i]) * V + picks[a + j]];
        }
    }
}

__global__ void k_gather_blk(uint32_t num_orders, const uint32_t *__restrict__ pick_off,
                             const uint32_t *__restrict__ picks,
                             const uint64_t *__restrict__ out_base,
                             const uint32_t *__restrict__ src_idx_of_pick, uint32_t lo, uint32_t n,
                             const uint32_t *__restrict__ dist, uint32_t V,
                             uint32_t *__restrict__ out) {
    for (uint32_t o = blockIdx.x; o < num_orders; o += gridDim.x) {
        const uint32_t a = pick_off[o], P = pick_off[o + 1] - a;
        const uint64_t ob = out_base[o];
        for (uint32_t k = threadIdx.x; k < P * P; k += blockDim.x) {
            const uint32_t i = k / P, j = k - i * P;
            const uint32_t si = src_idx_of_pick[a + i];
            if (si < lo || si >= lo + n) continue;
            const uint32_t c = si - lo;
            const size_t b = c / LANES, l = c % LANES;
            out[ob + k] = dist[(b * V + picks[a + j]) * LANES + l];
        }
    }
}

__global__ void k_gather_seg(uint32_t num_orders, const uint32_t *__restrict__ pick_off,
                             const uint32_t *__restrict__ picks,
                             const uint64_t *__restrict__ out_base,
                             const uint32_t *__restrict__ src_idx_of_pick, uint32_t lo, uint32_t n,
                             const uint32_t *__restrict__ tile_of, const uint32_t *__restrict__ pos_of,
                             const uint8_t *__restrict__ visited, const uint32_t *__restrict__ gdist,
                             uint32_t T, uint32_t Vt, uint32_t lanes_log2, uint32_t *__restrict__ out) {
    for (uint32_t o = blockIdx.x; o < num_orders; o += gridDim.x) {
        const uint32_t a = pick_off[o], P = pick_off[o + 1] - a;
        const uint64_t ob = out_base[o];
        for (uint32_t k = threadIdx.x; k < P * P; k += blockDim.x) {
            const uint32_t i = k / P, j = k - i * P;
            const uint32_t si = src_idx_of_pick[a + i];
            if (si < lo || si >= lo + n) continue;
            out[ob + k] = seg_value(tile_of, pos_of, visited, gdist, T, Vt, lanes_log2, si - lo,
                                    picks[a + i], picks[a + j]);
        }
    }
}

// ------------------------------------------------- canonical predecessors
// pred[r][v] = smallest u over in-arcs (u, v) with d(u) != INF and
// d(u) + w = d(v); -1 for the row's source and for INF vertices.
__global__ void k_pred_rows(const uint32_t *__restrict__ rows, uint32_t nrows, uint32_t V,
                            const uint32_t *__restrict__ row_src_vertex,
                            const uint32_t *__restrict__ in_ptr, const uint32_t *__restrict__ in_src,
                            const uint32_t *__restrict__ in_w, const uint32_t *__restrict__ in_row,
                            const uint32_t *__restrict__ out_row, int32_t *__restrict__ pred) {
    for (uint32_t r = blockIdx.y; r < nrows; r += gridDim.y) {
    const uint32_t *d = rows + static_cast<size_t>(in_row[r]) * V;
    int32_t *p = pred + static_cast<size_t>(out_row[r]) * V;
    const uint32_t sv = row_src_vertex[r];
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
        const uint32_t dv = d[v];
        int32_t best = -1;
        if (v != sv && dv != INF) {
            uint32_t bu = NONE;
            for (uint32_t e = in_ptr[v]; e < in_ptr[v + 1]; ++e) {
                const uint32_t u = in_src[e];
                const uint32_t du = d[u];
                if (du != INF && static_cast<uint64_t>(du) + in_w[e] == dv && u < bu) bu = u;
            }
            best = bu == NONE ? -1 : static_cast<int32_t>(bu);
        }
        p[v] = best;
    }
    }
}

// ------------------------------------------- paper-structured edge baseline
// One thread per arc (u, v, w), 256 threads per block; each thread loops
// over the N sources and lowers d_n(v) in place (the paper's one-thread-per-
// edge kernel over integer arrays u, v, w with dist of size V x N).
__global__ __launch_bounds__(256) void k_edge_round(const uint32_t *__restrict__ arc_src,
                                                    const uint32_t *__restrict__ col,
                                                    const uint32_t *__restrict__ w, uint32_t E,
                                                    uint32_t *__restrict__ dist, uint32_t V,
                                                    uint32_t N, uint32_t *__restrict__ changed) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const uint32_t u = arc_src[e], v = col[e], ww = w[e];
    bool moved = false;
    for (uint32_t n = 0; n < N; ++n) {
        uint32_t *dn = dist + static_cast<size_t>(n) * V;
        const uint32_t nd = sat_add(dn[u], ww);
        if (nd < dn[v]) moved |= nd < atomicMin(&dn[v], nd);
    }
    if (moved) *changed = 1u;
}

__global__ void k_rows_seed(uint32_t *__restrict__ dist, uint32_t V, uint32_t N,
                            const uint32_t *__restrict__ src) {
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) dist[static_cast<size_t>(n) * V + src[n]] = 0;
}

__global__ void k_arc_src(const uint32_t *__restrict__ row_ptr, uint32_t V,
                          uint32_t *__restrict__ arc_src) {
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < V; u += gridDim.x * blockDim.x)
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) arc_src[e] = u;
}

// ----------------------------------------------------------- weight epochs
__global__ void k_weight_scatter(uint32_t n, const uint32_t *__restrict__ arc,
                                 const uint32_t *__restrict__ neww, uint32_t *__restrict__ w,
                                 uint32_t *__restrict__ in_w, const uint32_t *__restrict__ in_pos,
                                 uint32_t *__restrict__ l_arc, uint32_t *__restrict__ x_w,
                                 const uint32_t *__restrict__ arc_slot, uint32_t *__restrict__ li_arc,
                                 const uint32_t *__restrict__ arc_slot_in) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t a = arc[i], nw = neww[i];
    w[a] = nw;
    in_w[in_pos[a]] = nw;
    if (arc_slot_in) {
        const uint32_t si = arc_slot_in[a];
        if (si != NONE) li_arc[si] = (li_arc[si] & 0xFFFF0000u) | (nw & 0xFFFFu);
    }
    if (arc_slot) {
        const uint32_t sl = arc_slot[a];
        if (sl == NONE) return;
        if (sl & 0x80000000u)
            x_w[sl & 0x7FFFFFFFu] = nw;
        else
            l_arc[sl] = (l_arc[sl] & 0xFFFF0000u) | (nw & 0xFFFFu);
    }
}

}  // namespace

// ========================================================== host launchers
void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st) {
    if (!n) return;
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (fill)");
    if ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)
        hipLaunchKernelGGL(k_fill_u32, blocks_for(n / 4 + 1, 256, 8192), 256, 0, st, p, n, v);
    else
        hipLaunchKernelGGL(k_fill_u32_unaligned, blocks_for(n, 256, 8192), 256, 0, st, p, n, v);
    check_launch("fill_u32");
}

void launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u8, blocks_for(n, 256, 8192), 256, 0, st, p, n, v);
    check_launch("fill_u8");
}

void launch_blk_seed(uint32_t *dist, uint32_t V, uint32_t S, const uint32_t *src, hipStream_t st) {
    if (!S) return;
    hipLaunchKernelGGL(k_blk_seed, blocks_for(S, 256), 256, 0, st, dist, V, S, src);
    check_launch("blk_seed");
}

void launch_sweep_pull(uint32_t *dist, uint32_t V, uint32_t nb, const uint32_t *in_ptr,
                       const uint32_t *in_src, const uint32_t *in_w, uint32_t *changed,
                       uint32_t grid, hipStream_t st) {
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (sweep)");
    hipLaunchKernelGGL(k_sweep_pull, grid, 256, 0, st, dist, V, nb, in_ptr, in_src, in_w, changed);
    check_launch("sweep_pull");
}

void launch_frontier_seed(uint64_t *list, uint32_t *count, uint32_t S, const uint32_t *src,
                          uint32_t V, hipStream_t st) {
    (void)V;
    hipLaunchKernelGGL(k_frontier_seed, blocks_for(S ? S : 1, 256), 256, 0, st, list, count, S, src);
    check_launch("frontier_seed");
}

void launch_frontier_push(uint32_t *dist, uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                          const uint32_t *w, const uint64_t *list_in, const uint32_t *count_in,
                          uint64_t *list_out, uint32_t *count_out, uint32_t *stamps,
                          const uint32_t *pass_ctr, uint32_t grid, hipStream_t st) {
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (frontier)");
    hipLaunchKernelGGL(k_frontier_push, grid, 256, 0, st, dist, V, row_ptr, col, w, list_in, count_in, list_out,
                                          count_out, stamps, pass_ctr);
    check_launch("frontier_push");
}

void launch_pass_prologue(uint32_t *count_next, const uint32_t *count_cur,
                          unsigned long long *stats, uint32_t *pass_ctr, hipStream_t st) {
    hipLaunchKernelGGL(k_pass_prologue, 1, 1, 0, st, count_next, count_cur, stats, pass_ctr);
    check_launch("pass_prologue");
}

void launch_blk_emit(const uint32_t *dist, uint32_t V, uint32_t rows, const uint32_t *row_src_idx,
                     const uint32_t *out_row, uint32_t *out, hipStream_t st) {
    if (!rows) return;
    dim3 grid(blocks_for(V, 256, 1024), rows < 65535u ? rows : 65535u);
    hipLaunchKernelGGL(k_blk_emit, grid, 256, 0, st, dist, V, rows, row_src_idx, out_row, out);
    check_launch("blk_emit");
}

static SegPassArgs seg_args(const TileSet &ts, const SegState &ss, uint32_t par, uint32_t G) {
    SegPassArgs A{};
    A.tile_base = ts.d_tile_base.p;
    A.l_off = ts.d_l_off.p;
    A.l_arc = ts.d_l_arc.p;
    A.x_off = ts.d_x_off.p;
    A.x_port = ts.d_x_port.p;
    A.x_w = ts.d_x_w.p;
    A.x_tile = ts.d_x_tile.p;
    A.port_base = ts.d_port_base.p;
    A.port_local = ts.d_port_local.p;
    A.bo_base = ts.d_bo_base.p;
    A.bo_local = ts.d_bo_local.p;
    A.T = ts.T;
    A.Vt = ts.Vt;
    A.NP = ts.NP;
    A.S = ss.S;
    A.gdist = ss.gdist;
    A.inbox = ss.inbox;
    A.visited = ss.visited;
    A.stamps = ss.stamps;
    A.src_pos = ss.src_pos;
    A.src_tile = ss.src_tile;
    const uint32_t nx = par ^ 1u;
    A.cnt_cur = ss.cnt + static_cast<size_t>(par) * ts.T;
    A.bucket_cur = ss.bucket + static_cast<size_t>(par) * ts.T * ss.S;
    A.cnt_next = ss.cnt + static_cast<size_t>(nx) * ts.T;
    A.bucket_next = ss.bucket + static_cast<size_t>(nx) * ts.T * ss.S;
    A.tiles_next = ss.tiles + static_cast<size_t>(nx) * ts.T;
    A.ntiles_next = ss.ntiles + nx;
    A.units = ss.units;
    A.flags = ss.flags;
    A.xval = ss.xval;
    A.NB = ts.NB;
    A.pin_off = ts.d_pin_off.p;
    A.pin_rec = ts.d_pin_rec.p;
    A.hdr2 = reinterpret_cast<const uint2 *>(ts.d_ovl_hdr2.p);
    A.nunits = ss.nunits;
    A.cursor = ss.cursor;
    A.pass_ctr = ss.pass_ctr;
    A.G = G;
    A.li_off = ts.d_li_off.p;
    A.li_arc = ts.d_li_arc.p;
    A.nsrc = ss.nsrc;
    A.tile_visits = ss.tile_visits;
    A.wave_stores = ss.wave_stores;
    return A;
}

void launch_seg_seed_n(const TileSet &ts, const SegState &ss, uint32_t n, hipStream_t st) {
    // seeds land in parity 0; their stamp is 1 (pass 0's list)
    SegPassArgs A = seg_args(ts, ss, 1u, 1u);
    A.flags = nullptr;
    hipLaunchKernelGGL(k_seg_seed, blocks_for(n ? n : 1, 256), 256, 0, st, A, n, ss.lanes_log2);
    check_launch("seg_seed");
}

void launch_seg_step(const TileSet &ts, const SegState &ss, uint32_t par, uint32_t tile_cap,
                     uint32_t waves, uint32_t G, uint32_t grid, hipStream_t st, hipEvent_t ev_begin,
                     hipEvent_t ev_end) {
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (segment pass)");
    const uint32_t nx = par ^ 1u;
    hipLaunchKernelGGL(k_seg_prologue, blocks_for(ts.T, 256, 64), 256, 0, st, 
        ss.cnt + static_cast<size_t>(nx) * ts.T, ts.T, ss.ntiles + nx, ss.nunits, ss.cursor,
        ss.pass_ctr);
    check_launch("seg_prologue");
    hipLaunchKernelGGL(k_seg_plan, blocks_for(ts.T, 256, 64), 256, 0, st, 
        ss.tiles + static_cast<size_t>(par) * ts.T, ss.ntiles + par,
        ss.cnt + static_cast<size_t>(par) * ts.T, G, ss.units, ss.nunits, ss.stats);
    check_launch("seg_plan");
    SegPassArgs A = seg_args(ts, ss, par, G);
    if (ss.lanes_log2 == 6) {
#define WR_SEGB_CASE(CAPV, NWV)                                                          \
        if (tile_cap == CAPV && waves == NWV) {                                          \
            if (ev_begin) WR_HIP(hipEventRecord(ev_begin, st));                          \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_segb_pass<CAPV, NWV>), grid, NWV * 64, 0, st, A); \
            check_launch("segb_pass");                                                   \
            if (ev_end) WR_HIP(hipEventRecord(ev_end, st));                              \
            return;                                                                      \
        }
        WR_SEGB_CASE(256, 8)
        WR_SEGB_CASE(256, 16)
        WR_SEGB_CASE(512, 8)
        WR_SEGB_CASE(512, 16)
#undef WR_SEGB_CASE
        fail(WR_E_UNSUPPORTED, "no source-blocked segment kernel for tile size " +
                                   std::to_string(tile_cap) + " with " + std::to_string(waves) + " waves");
    }
#define WR_SEG_CASE(CAPV, NWV)                                                           \
    if (tile_cap == CAPV && waves == NWV) {                                              \
        if (ev_begin) WR_HIP(hipEventRecord(ev_begin, st));                              \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_seg_pass<CAPV, NWV>), grid, NWV * 64, 0, st, A); \
        check_launch("seg_pass");                                                        \
        if (ev_end) WR_HIP(hipEventRecord(ev_end, st));                                  \
        return;                                                                          \
    }
    WR_SEG_CASE(1024, 4)
    WR_SEG_CASE(1024, 8)
    WR_SEG_CASE(2048, 4)
    WR_SEG_CASE(2048, 8)
    WR_SEG_CASE(4096, 2)
#undef WR_SEG_CASE
    fail(WR_E_UNSUPPORTED, "no segment kernel for tile size " + std::to_string(tile_cap) +
                               " with " + std::to_string(waves) + " waves");
}

uint32_t seg_pass_lds_bytes(uint32_t tile_cap, uint32_t waves, uint32_t lanes) {
    const uint32_t words = tile_cap / 32;
    if (lanes == 64)
        return tile_cap * 256 + 2 * tile_cap * 4 + 4 * tile_cap * (4 + 2) + 3 * words * 4 +
               tile_cap * 2 + 8;
    return (tile_cap + 2) * 2 + 4 * tile_cap * 4 +
           waves * (tile_cap * 4 + tile_cap * 2 + 2 * words * 4) + 4;
}

void launch_seg_emit(const TileSet &ts, const SegState &ss, uint32_t V, uint32_t rows,
                     const uint32_t *row_src_idx, const uint32_t *row_src_vertex,
                     const uint32_t *out_row, uint32_t *out, hipStream_t st) {
    if (!rows) return;
    dim3 grid(blocks_for(V, 256, 1024), rows < 65535u ? rows : 65535u);
    hipLaunchKernelGGL(k_seg_emit, grid, 256, 0, st, ts.d_tile_of.p, ts.d_pos_of.p, ss.visited, ss.gdist,
                       ts.T, ts.Vt, ss.lanes_log2, V, rows, row_src_idx, row_src_vertex, out_row, out);
    check_launch("seg_emit");
}

void launch_gather_rows(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                        const uint64_t *out_base, const uint32_t *row_of_pick, const uint32_t *rows,
                        uint32_t V, uint32_t *out, hipStream_t st) {
    if (!num_orders) return;
    hipLaunchKernelGGL(k_gather_rows, blocks_for(num_orders, 1, 65535), 256, 0, st, 
        num_orders, pick_off, picks, out_base, row_of_pick, rows, V, out);
    check_launch("gather_rows");
}

void launch_gather_blk(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                       const uint64_t *out_base, const uint32_t *src_idx_of_pick, uint32_t chunk_lo,
                       uint32_t chunk_n, const uint32_t *dist, uint32_t V, uint32_t *out,
                       hipStream_t st) {
    if (!num_orders) return;
    hipLaunchKernelGGL(k_gather_blk, blocks_for(num_orders, 1, 65535), 256, 0, st, 
        num_orders, pick_off, picks, out_base, src_idx_of_pick, chunk_lo, chunk_n, dist, V, out);
    check_launch("gather_blk");
}

void launch_gather_seg(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                       const uint64_t *out_base, const uint32_t *src_idx_of_pick, uint32_t chunk_lo,
                       uint32_t chunk_n, const TileSet &ts, const SegState &ss, uint32_t *out,
                       hipStream_t st) {
    if (!num_orders) return;
    hipLaunchKernelGGL(k_gather_seg, blocks_for(num_orders, 1, 65535), 256, 0, st, 
        num_orders, pick_off, picks, out_base, src_idx_of_pick, chunk_lo, chunk_n, ts.d_tile_of.p,
        ts.d_pos_of.p, ss.visited, ss.gdist, ts.T, ts.Vt, ss.lanes_log2, out);
    check_launch("gather_seg");
}

void launch_pred_rows(const uint32_t *rows, uint32_t nrows, uint32_t V, const uint32_t *row_src_vertex,
                      const uint32_t *in_ptr, const uint32_t *in_src, const uint32_t *in_w,
                      const uint32_t *in_row, const uint32_t *out_row, int32_t *pred, hipStream_t st) {
    if (!nrows) return;
    dim3 grid(blocks_for(V, 256, 1024), nrows < 65535u ? nrows : 65535u);
    hipLaunchKernelGGL(k_pred_rows, grid, 256, 0, st, rows, nrows, V, row_src_vertex, in_ptr, in_src, in_w, in_row,
                                       out_row, pred);
    check_launch("pred_rows");
}

void launch_edge_round(const uint32_t *arc_src, const uint32_t *col, const uint32_t *w, uint32_t E,
                       uint32_t *dist, uint32_t V, uint32_t N, uint32_t *changed, hipStream_t st) {
    if (!E) return;
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (edge round)");
    hipLaunchKernelGGL(k_edge_round, (E + 255) / 256, 256, 0, st, arc_src, col, w, E, dist, V, N, changed);
    check_launch("edge_round");
}

void launch_rows_seed(uint32_t *dist, uint32_t V, uint32_t N, const uint32_t *src, hipStream_t st) {
    if (!N) return;
    hipLaunchKernelGGL(k_rows_seed, blocks_for(N, 256), 256, 0, st, dist, V, N, src);
    check_launch("rows_seed");
}

void launch_arc_src(const uint32_t *row_ptr, uint32_t V, uint32_t *arc_src, hipStream_t st) {
    hipLaunchKernelGGL(k_arc_src, blocks_for(V, 256, 4096), 256, 0, st, row_ptr, V, arc_src);
    check_launch("arc_src");
}

void launch_weight_scatter(uint32_t n, const uint32_t *arc, const uint32_t *neww, uint32_t *w,
                           uint32_t *in_w, const uint32_t *in_pos, uint32_t *l_arc, uint32_t *x_w,
                           const uint32_t *arc_slot, uint32_t *li_arc, const uint32_t *arc_slot_in,
                           hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_weight_scatter, blocks_for(n, 256), 256, 0, st, n, arc, neww, w, in_w, in_pos,
                       l_arc, x_w, arc_slot, li_arc, arc_slot_in);
    check_launch("weight_scatter");
}

void launch_ovl_custom(const TileSet &ts, uint32_t tile_cap, uint32_t *F, uint32_t grid, hipStream_t st,
                       bool reverse) {
    SegState dummy;
    SegPassArgs A = seg_args(ts, dummy, 0u, 1u);
#define WR_CUSTOM_CASE(CAPV)                                                                          \
    if (tile_cap == CAPV) {                                                                           \
        if (reverse)                                                                                  \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ovl_custom<CAPV, 8, true>), grid, 512, 0, st, A, F);  \
        else                                                                                          \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ovl_custom<CAPV, 8, false>), grid, 512, 0, st, A, F); \
        check_launch("ovl_custom");                                                                   \
        return;                                                                                       \
    }
    WR_CUSTOM_CASE(256)
    WR_CUSTOM_CASE(512)
#undef WR_CUSTOM_CASE
    fail(WR_E_UNSUPPORTED, "overlay tables need tiles of at most 512 vertices");
}

// most exits, table columns (incoming cross arcs, rounded up to 4) and
// cross arcs leaving or entering one tile
static void ovl_dims(const TileSet &ts, uint32_t &XM, uint32_t &EM, uint32_t &PM) {
    XM = std::max(ts.max_exits, 1u);
    EM = (std::max(ts.max_cross_in, 1u) + 3u) / 4u * 4u;
    PM = std::max(std::max(ts.max_cross, ts.max_cross_in), 1u);
}

uint32_t ovl_row_entries(const TileSet &ts) {
    uint32_t XM, EM, PM;
    ovl_dims(ts, XM, EM, PM);
    return EM;
}

uint32_t ovl_pass_lds_bytes(const TileSet &ts) {
    uint32_t XM, EM, PM;
    ovl_dims(ts, XM, EM, PM);
    return (XM * EM + 2 * EM * 64 + XM + 1 + 3 * PM + 1) * 4;
}

__global__ void k_ovl_pin_rec(uint2 *__restrict__ rec, const uint32_t *__restrict__ pin_xa,
                              const uint32_t *__restrict__ pin_exit, const uint32_t *__restrict__ pin_lport,
                              const uint32_t *__restrict__ x_w, uint32_t n) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
        rec[k] = make_uint2(pin_exit[k], (x_w[pin_xa[k]] & 0xFFFFu) | (pin_lport[k] << 16));
}

void launch_ovl_pin_rec(const TileSet &ts, hipStream_t st) {
    const uint32_t n = static_cast<uint32_t>(ts.pin_xa.size());
    if (!n) return;
    hipLaunchKernelGGL(k_ovl_pin_rec, blocks_for(n, 256, 4096), 256, 0, st, ts.d_pin_rec.p, ts.d_pin_xa.p,
                       ts.d_pin_exit.p, ts.d_pin_lport.p, ts.d_x_w.p, n);
    check_launch("ovl_pin_rec");
}

void launch_ovl_pack(const TileSet &ts, hipStream_t st) {
    hipLaunchKernelGGL(k_ovl_pack, blocks_for(ts.T, 4, 4096), 256, 0, st, ts.d_F.p, ts.d_tile_base.p,
                       ts.d_bo_local.p, reinterpret_cast<const uint4 *>(ts.d_ovl_hdr.p),
                       reinterpret_cast<const uint2 *>(ts.d_ovl_hdr2.p), ts.d_pin_lport.p, ts.T, ts.ovl_em,
                       ts.d_Fx.p);
    check_launch("ovl_pack");
}

// The overlay steps keep the unit count and cursor per parity (parity 0 in
// nunits[0] / cursor[0], parity 1 three words further), so a step's plan
// can zero the next step's pair while its own pass runs on the current one.
void launch_ovl_step(const TileSet &ts, const SegState &ss, uint32_t par, uint32_t G, uint32_t grid,
                     const uint32_t *F, bool count_after, hipStream_t st, hipEvent_t ev_begin,
                     hipEvent_t ev_end, const uint32_t *bound) {
    (void)F;
    if (fault_launch_now()) fail(WR_E_DEVICE, "injected launch failure (overlay pass)");
    const uint32_t nx = par ^ 1u;
    uint32_t *nunits_cur = ss.nunits + 3u * par, *cursor_cur = ss.cursor + 3u * par;
    uint32_t *nunits_nx = ss.nunits + 3u * nx, *cursor_nx = ss.cursor + 3u * nx;
    hipLaunchKernelGGL(k_ovl_plan, blocks_for(ts.T, OVL_PLAN_WAVES, 1024), OVL_PLAN_WAVES * 64, 0, st, ss.flags,
                       ts.T, ss.S,
                       ss.cnt + static_cast<size_t>(par) * ts.T, ss.bucket + static_cast<size_t>(par) * ts.T * ss.S,
                       G, ss.units, nunits_cur, nunits_nx, cursor_nx, ss.ntiles + nx, ss.pending, ss.stats,
                       ss.tile_visits);
    check_launch("ovl_plan");
    SegPassArgs A = seg_args(ts, ss, par, G);
    A.nunits = nunits_cur;
    A.cursor = cursor_cur;
    A.bound = bound;
    uint32_t XM, EM, PM;
    ovl_dims(ts, XM, EM, PM);
    const uint32_t lds = ovl_pass_lds_bytes(ts);
    const uint4 *hd = reinterpret_cast<const uint4 *>(ts.d_ovl_hdr.p);
    if (ev_begin) WR_HIP(hipEventRecord(ev_begin, st));
    // rows (and exits) per wave: the smallest instance covering the tiling
    const uint32_t need = (std::max(XM, EM) + OVL_NW - 1) / OVL_NW;
#define WR_OVL_PASS(RR)                                                                                  \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_ovl_pass<OVL_NW, RR>), grid, OVL_NW * 64, lds, st, A, ts.d_Fx.p, \
                       hd, ts.d_bo_xbeg.p, XM, EM, PM)
    if (need <= 4) WR_OVL_PASS(4);
    else if (need <= 5) WR_OVL_PASS(5);
    else if (need <= 6) WR_OVL_PASS(6);
    else WR_OVL_PASS(8);
#undef WR_OVL_PASS
    check_launch("ovl_pass");
    if (ev_end) WR_HIP(hipEventRecord(ev_end, st));
    if (count_after) {
        const size_t n = static_cast<size_t>(ts.T) * ss.S;
        hipLaunchKernelGGL(k_flags_any, blocks_for(n, 256, 512), 256, 0, st, ss.flags, n, ss.S, ss.ntiles + nx,
                           ss.pending);
        check_launch("flags_any");
    }
}

static OvlRead ovl_read(const TileSet &ts, const SegState &ss, const uint32_t *F) {
    OvlRead R{};
    R.tile_of = ts.d_tile_of.p;
    R.pos_of = ts.d_pos_of.p;
    R.hdr2 = reinterpret_cast<const uint2 *>(ts.d_ovl_hdr2.p);
    R.pin_rec = ts.d_pin_rec.p;
    R.xval = ss.xval;
    R.F = F;
    R.NB = ts.NB;
    return R;
}

void launch_ovl_emit(const TileSet &ts, const SegState &ss, const uint32_t *F, uint32_t V, uint32_t rows,
                     const uint32_t *row_src_vertex, const uint32_t *out_row, const uint32_t *grp_block,
                     const uint32_t *lane_row, uint32_t ngroups, uint32_t num_cus, uint32_t *out, hipStream_t st) {
    if (!rows) return;
    dim3 fgrid(blocks_for(V, 256, 1024), rows < 65535u ? rows : 65535u);
    hipLaunchKernelGGL(k_fill_rows, fgrid, 256, 0, st, out, V, rows, out_row, INF);
    check_launch("fill_rows");
    const uint64_t items = static_cast<uint64_t>(ts.T) * ngroups;
    if (items) {
        const uint32_t lds = (64u + ROWS_NW * ROWS_CHUNK * 65u + std::max(ts.max_ports, 1u) * 64u) * 4u;
        const uint32_t grid = static_cast<uint32_t>(std::min<uint64_t>(items, static_cast<uint64_t>(num_cus) * 16u));
        hipLaunchKernelGGL(k_ovl_rows, grid, ROWS_NW * 64, lds, st, ovl_read(ts, ss, F), ts.d_tile_base.p,
                           reinterpret_cast<const uint4 *>(ts.d_ovl_hdr.p), ts.T, grp_block, lane_row, items,
                           ts.d_vert_of.p, V, out);
        check_launch("ovl_rows");
    }
    hipLaunchKernelGGL(k_rows_src_zero, blocks_for(rows, 256, 1024), 256, 0, st, out, V, rows, out_row,
                       row_src_vertex);
    check_launch("rows_src_zero");
}

void launch_bound_refine(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                         const uint32_t *src_idx_of_pick, uint32_t chunk_lo, uint32_t chunk_n, const TileSet &ts,
                         const SegState &ss, const uint32_t *F, uint32_t *bound, uint32_t *tmp, hipStream_t st) {
    if (!num_orders || !chunk_n) return;
    dim3 grid(std::min(num_orders, 65535u), 4);
    hipLaunchKernelGGL(k_bound_pairs, grid, 256, 0, st, num_orders, pick_off, picks, src_idx_of_pick, chunk_lo,
                       chunk_n, ovl_read(ts, ss, F), tmp);
    check_launch("bound_pairs");
    hipLaunchKernelGGL(k_bound_min, blocks_for(chunk_n, 256, 1024), 256, 0, st, bound, tmp, chunk_n);
    check_launch("bound_min");
}

void launch_gather_ovl(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *picks,
                       const uint64_t *out_base, const uint32_t *src_idx_of_pick, uint32_t chunk_lo,
                       uint32_t chunk_n, const TileSet &ts, const SegState &ss, const uint32_t *F,
                       uint32_t *out, hipStream_t st) {
    if (!num_orders) return;
    // four workgroups per order: one pair per thread for orders of up to 32
    // picks, larger orders loop
    dim3 grid(std::min(num_orders, 65535u), 4);
    hipLaunchKernelGGL(k_gather_ovl, grid, 256, 0, st, num_orders, pick_off, picks, out_base, src_idx_of_pick,
                       chunk_lo, chunk_n, ovl_read(ts, ss, F), out);
    check_launch("gather_ovl");
}

void launch_ovl_seed_push(const TileSet &ts, const SegState &ss, const uint32_t *slots, uint32_t nslots,
                          hipStream_t st) {
    if (!nslots) return;
    SegPassArgs A = seg_args(ts, ss, 0u, 1u);
    hipLaunchKernelGGL(k_ovl_seed_push, blocks_for(nslots, 4, 4096), 256, 0, st, A, ts.d_B.p,
                       reinterpret_cast<const uint4 *>(ts.d_ovl_hdr.p), ts.d_bo_xbeg.p, slots, nslots);
    check_launch("ovl_seed_push");
}

void IntileJob::upload_and_launch(wr_context *ctx, const TileSet &ts, const IntileWork &w, bool full, uint32_t V,
                                  uint32_t *out, hipStream_t st) {
    ng = static_cast<uint32_t>(w.grp.size() / 4);
    npairs = static_cast<uint32_t>(w.pair_key.size());
    if (!ng) return;
    upload_reuse(d_grp, ctx, w.grp, st);
    upload_reuse(d_src, ctx, w.src_local, st);
    if (full) {
        upload_reuse(d_row, ctx, w.row, st);
    } else {
        upload_reuse(d_key, ctx, w.pair_key, st);
        upload_reuse(d_out, ctx, w.pair_out, st);
        if (!out) reserve(d_val, ctx, npairs);
    }
    SegState dummy;
    SegPassArgs A = seg_args(ts, dummy, 0u, 1u);
    const IntileGroup *G = reinterpret_cast<const IntileGroup *>(d_grp.p);
    const uint32_t grid = std::min<uint32_t>(ng, 4096u);
    uint32_t *val = (!full && !out) ? d_val.p : nullptr;
    if (ts.tile_cap == 256)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_intile_fix<256, 8>), grid, 512, 0, st, A, G, ng, d_src.p,
                           full ? nullptr : d_key.p, full ? nullptr : d_out.p, full ? d_row.p : nullptr,
                           ts.d_vert_of.p, V, out, val);
    else if (ts.tile_cap == 512)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_intile_fix<512, 8>), grid, 512, 0, st, A, G, ng, d_src.p,
                           full ? nullptr : d_key.p, full ? nullptr : d_out.p, full ? d_row.p : nullptr,
                           ts.d_vert_of.p, V, out, val);
    else
        fail(WR_E_UNSUPPORTED, "in-tile fix-up needs tiles of at most 512 vertices");
    check_launch("intile_fix");
}

void IntileJob::apply(uint32_t *out, hipStream_t st) const {
    if (!npairs || !d_val.p) return;
    hipLaunchKernelGGL(k_min_scatter, blocks_for(npairs, 256, 1024), 256, 0, st, d_out.p, d_val.p, npairs, out);
    check_launch("min_scatter");
}

void launch_intile_fix(wr_context *ctx, const TileSet &ts, const IntileWork &w, bool full, uint32_t V,
                       uint32_t *out, hipStream_t st) {
    IntileJob job;
    job.upload_and_launch(ctx, ts, w, full, V, out, st);
    if (job.ng) WR_HIP(hipStreamSynchronize(st));   // the uploaded tables are freed on return
}

uint32_t ovl_max_exits() { return OVL_XCAP; }
uint32_t ovl_max_cross() { return OVL_PCAP; }
uint32_t ovl_max_entries() { return OVL_ECAP; }
uint32_t ovl_waves() { return OVL_NW; }


// ------------------------------------------------------------ order routes
// Optimal open route over each order's stops (Route Optimization section:
// an ordering of the P stops with free ends, length = sum of its P-1 matrix
// steps), by Held and Karp's programme over stop subsets, which that section
// names as the exact alternative to enumerating orderings:
//   h(S, i) = shortest path that starts at stop i and visits exactly S,
//   h({i}, i) = 0,  h(S, i) = min_{j in S\{i}} D[i][j] + h(S\{i}, j).
// One workgroup per order keeps the matrix and every state in LDS: only the
// states with i in S exist, P * 2^(P-1) words, state (S, i) at
// sbase(S) + |S below i| where sbase(S) = sum of |T| over T < S.  Subsets are
// processed layer by layer (|S| = 2..P, a barrier between layers); a thread
// takes one state at a time: a per-order table lists the subsets by size
// (each at its layer's start plus its colex rank among subsets of that
// size), so the thread's item index gives the subset with one lookup, i is
// the subset's m-th member, and the minimum runs over the members of S\{i}
// only.  Lengths accumulate in 32
// bits with WR_INF absorbing; a finite sum that would reach WR_INF raises
// *overflow and the call fails.  The route is read greedily by one thread:
// the smallest first stop that reaches the optimum, then repeatedly the
// smallest next stop whose step keeps it, which is the lexicographically
// smallest shortest ordering.
constexpr uint32_t RT_NMAX = 12;
constexpr uint32_t RT_THREADS = 1024;

// number of stops summed over all subsets T < S (n <= 31)
__device__ __forceinline__ uint32_t rt_sbase(uint32_t S, uint32_t n) {
    uint32_t t = 0;
    for (uint32_t b = 0; b < n; ++b) {
        t += (S >> (b + 1)) << b;
        const uint32_t r = S & ((2u << b) - 1u);
        t += r > (1u << b) ? r - (1u << b) : 0u;
    }
    return t;
}

__device__ __forceinline__ uint32_t rt_step(uint32_t h, uint32_t d, bool &ovf) {
    // branch-free: INF absorbs; a finite sum reaching INF flags the overflow
    const uint32_t s = h + d;
    const bool inf = h == INF || d == INF;
    const bool wrap = !inf && (s < h || s == INF);
    ovf = ovf || wrap;
    return (inf || wrap) ? INF : s;
}

// LDS layout of one subset programme: binomials, the matrix, subset offsets,
// subsets by size and the states (nmax = largest n the launch serves)
struct RtLds {
    uint32_t *bin, *D, *base, *ord, *H;
};
constexpr uint32_t RT_BIN_WORDS = ((RT_NMAX + 1) * (RT_NMAX + 1) + 1) & ~1u;   // even: later arrays stay 8-aligned
__device__ __forceinline__ RtLds rt_layout(uint32_t *lds, uint32_t nmax) {
    RtLds L;
    L.bin = lds;                                     // [(RT_NMAX+1)^2] C(c, t)
    L.D = L.bin + RT_BIN_WORDS;                      // [nmax * nmax]
    L.base = L.D + nmax * nmax;                      // [2^nmax]
    L.ord = L.base + (1u << nmax);                   // [2^nmax] subsets by size, colex within a size
    L.H = L.ord + (1u << nmax);                      // [nmax * 2^(nmax-1)]
    return L;
}
__host__ __device__ constexpr uint32_t rt_lds_words(uint32_t nmax) {
    return RT_BIN_WORDS + nmax * nmax + 2u * (1u << nmax) + nmax * (1u << (nmax ? nmax - 1 : 0));
}

// binomial table; the caller synchronises before its first use
__device__ void rt_binomials(uint32_t *bin) {
    constexpr uint32_t NB1 = RT_NMAX + 1;
    for (uint32_t q = threadIdx.x; q < NB1 * NB1; q += blockDim.x) {
        const uint32_t c = q / NB1, t = q % NB1;
        uint32_t v = t <= c ? 1u : 0u;   // C(c, t) by the product formula
        for (uint32_t x = 1; x <= t && t <= c; ++x) v = v * (c - t + x) / x;
        bin[q] = v;
    }
}

// Subset offsets and subsets by size for n elements (1 <= n <= RT_NMAX), by
// the whole workgroup; ends synchronised.
__device__ void rt_tables(const RtLds &L, uint32_t n) {
    constexpr uint32_t NB1 = RT_NMAX + 1;
    const uint32_t nsub = 1u << n;
    for (uint32_t S = threadIdx.x; S < nsub; S += blockDim.x) {
        L.base[S] = rt_sbase(S, n);
        // subsets smaller than |S|, then S's colex rank among its size
        const uint32_t k = __builtin_popcount(S);
        uint32_t pos = 0;
        for (uint32_t x = 0; x < k; ++x) pos += L.bin[n * NB1 + x];
        uint32_t t = 1;
        for (uint32_t U = S; U != 0; U &= U - 1u, ++t) pos += L.bin[__builtin_ctz(U) * NB1 + t];
        L.ord[pos] = S;
    }
    __syncthreads();
}

// The states h(S, i) of the n x n matrix already in L.D (1 <= n <= RT_NMAX),
// by the whole workgroup, with the subset tables of n already in L (see
// rt_tables); ends synchronised.
__device__ void rt_solve(const RtLds &L, uint32_t n, bool &ovf) {
    constexpr uint32_t NB1 = RT_NMAX + 1;
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < n; i += blockDim.x) L.H[L.base[1u << i]] = 0u;
    __syncthreads();
    uint32_t lstart = 1 + n;   // the empty set and the singletons come first
    for (uint32_t k = 2; k <= n; ++k) {
        const uint32_t items = L.bin[n * NB1 + k] * k;
        for (uint32_t q = tid; q < items; q += blockDim.x) {
            const uint32_t r = q / k, m = q - r * k;
            const uint32_t S = L.ord[lstart + r];
            uint32_t T = S;
            for (uint32_t x = 0; x < m; ++x) T &= T - 1u;
            const uint32_t i = __builtin_ctz(T);
            const uint32_t R = S & ~(1u << i);
            const uint32_t bR = L.base[R];
            const uint32_t *Di = L.D + i * n;
            // the members j of R in ascending order, with h(R, j) at
            // consecutive states; two candidates per step keep two LDS
            // reads of each kind in flight
            uint32_t best = INF, rj = 0;
            uint32_t U = R;
            for (; U != 0 && (U & (U - 1u)) != 0; rj += 2) {
                const uint32_t j0 = __builtin_ctz(U);
                U &= U - 1u;
                const uint32_t j1 = __builtin_ctz(U);
                U &= U - 1u;
                const uint32_t c0 = rt_step(L.H[bR + rj], Di[j0], ovf);
                const uint32_t c1 = rt_step(L.H[bR + rj + 1], Di[j1], ovf);
                best = min(best, min(c0, c1));
            }
            if (U != 0) best = min(best, rt_step(L.H[bR + rj], Di[__builtin_ctz(U)], ovf));
            L.H[L.base[S] + m] = best;
        }
        lstart += L.bin[n * NB1 + k];
        __syncthreads();
    }
}

// One thread: the lexicographically smallest shortest ordering into route[],
// returning its length (INF when none is finite).
__device__ uint32_t rt_read_route(const RtLds &L, uint32_t n, uint32_t *route) {
    const uint32_t all = (1u << n) - 1u, bA = L.base[all];
    uint32_t opt = INF;
    for (uint32_t i = 0; i < n; ++i) opt = min(opt, L.H[bA + i]);
    uint32_t cur = 0;
    while (L.H[bA + cur] != opt) ++cur;
    uint32_t S = all;
    route[0] = cur;
    for (uint32_t k = 1; k < n; ++k) {
        const uint32_t hS = L.H[L.base[S] + __builtin_popcount(S & ((1u << cur) - 1u))];
        const uint32_t R = S & ~(1u << cur);
        const uint32_t bR = L.base[R];
        uint32_t nxt = 0, rj = 0;
        bool dummy = false;
        for (uint32_t j = 0; j < n; ++j) {
            if (!((R >> j) & 1u)) continue;
            if (rt_step(L.H[bR + rj], L.D[cur * n + j], dummy) == hS) {
                nxt = j;
                break;
            }
            ++rj;
        }
        route[k] = nxt;
        S = R;
        cur = nxt;
    }
    return opt;
}

__global__ __launch_bounds__(RT_THREADS) void k_route_hk(uint32_t num_orders, const uint32_t *__restrict__ off,
                                                         const uint64_t *__restrict__ mbase,
                                                         const uint32_t *__restrict__ dist,
                                                         uint64_t *__restrict__ len_out,
                                                         uint32_t *__restrict__ route_out,
                                                         uint32_t *__restrict__ overflow, uint32_t nmax) {
    HIP_DYNAMIC_SHARED(uint32_t, lds)
    const RtLds L = rt_layout(lds, nmax);
    const uint32_t tid = threadIdx.x;
    rt_binomials(L.bin);
    __syncthreads();   // the table is read by every thread from here on
    uint32_t tab_n = 0;   // stops the subset tables in LDS were built for
    for (uint32_t o = blockIdx.x; o < num_orders; o += gridDim.x) {
        const uint32_t a = off[o], n = off[o + 1] - a;
        if (n == 0) {
            if (tid == 0) len_out[o] = 0;
            continue;
        }
        const uint32_t *Dg = dist + mbase[o];
        for (uint32_t q = tid; q < n * n; q += blockDim.x) L.D[q] = Dg[q];
        if (n != tab_n) {
            rt_tables(L, n);   // synchronises (the matrix is then in LDS too)
            tab_n = n;
        } else {
            __syncthreads();
        }
        bool ovf = false;
        rt_solve(L, n, ovf);
        if (ovf) atomicOr(overflow, 1u);
        if (tid == 0) {
            const uint32_t opt = rt_read_route(L, n, route_out + a);
            len_out[o] = opt == INF ? ~0ull : static_cast<uint64_t>(opt);
        }
        __syncthreads();   // the next order reuses the LDS
    }
}

// ------------------------------------------------- cluster-decomposed route
// The route of the Route Optimization section's theorem: the order's stops
// are clustered by K-means on their positions (a cluster's centre is the
// mean position of its picks), each cluster gets its optimal open route,
// and the global route is the cheapest chaining of the cluster routes over
// every order of the clusters and every orientation of each.  Readings
// where the section is silent (shared with the oracle): integer positions,
// squared distances to a centre sum/c compared exactly as
// |c p - sum|^2 times the other cluster's c^2 (64-bit: |x|, |y| < 2^16,
// n <= 64); farthest-point initial centres from the first pick, ties to the
// smaller index; Lloyd steps until no assignment changes (at most 100),
// ties to the smaller cluster, an empty cluster keeping its centre; m grows
// by one while some cluster has more than RT_NMAX picks; among the cheapest
// chains the lexicographically smallest sequence of (cluster, orientation)
// wins, forward before reversed.
//
// One workgroup per order: wave 0 runs K-means with a lane per pick, the
// whole workgroup runs each cluster's subset programme, then a second
// subset programme over the K non-empty clusters chains them:
// g(S, c, o) = the cheapest chain that starts with cluster c in
// orientation o and uses exactly the clusters of S, g({c}, c, o) = len(c, o),
// g(S, c, o) = len(c, o) + min over c' in S\{c}, o' of
// D[end(c, o)][start(c', o')] + g(S\{c}, c', o') -- the minimum over every
// order and orientation, in 2 K 2^(K-1) states that reuse the LDS of the
// per-cluster states.
constexpr uint32_t RC_NMAX = 64;   // stops per order
constexpr uint32_t RC_MMAX = 10;   // clusters: 2 * 10 * 2^9 chain states fit the state area
constexpr uint32_t RC_ERR_RANGE = 1u, RC_ERR_CLUSTER = 2u;

__global__ __launch_bounds__(RT_THREADS) void k_route_clustered(
    uint32_t num_orders, const uint32_t *__restrict__ off, const uint64_t *__restrict__ mbase,
    const uint32_t *__restrict__ dist, const int32_t *__restrict__ xy, uint32_t m0,
    uint64_t *__restrict__ len_out, uint32_t *__restrict__ route_out, uint32_t *__restrict__ m_out,
    uint32_t *__restrict__ err) {
    HIP_DYNAMIC_SHARED(uint32_t, lds)
    const RtLds L = rt_layout(lds, RT_NMAX);
    uint32_t *sF = L.H + RT_NMAX * (1u << (RT_NMAX - 1));   // [RC_NMAX^2] the order's matrix
    int32_t *sXY = reinterpret_cast<int32_t *>(sF + RC_NMAX * RC_NMAX);   // [2 RC_NMAX]
    uint32_t *sAsg = reinterpret_cast<uint32_t *>(sXY + 2 * RC_NMAX);     // [RC_NMAX] cluster of each pick
    uint32_t *sRoute = sAsg + RC_NMAX;          // [RC_NMAX] cluster routes, concatenated (pick indices)
    uint32_t *sCl = sRoute + RC_NMAX;           // [RC_MMAX][4]: start in sRoute, size, forward, reverse length
    uint32_t *sMisc = sCl + 4 * RC_MMAX;        // [4]: clusters used, non-empty clusters, flags
    int64_t *sCen = reinterpret_cast<int64_t *>(sMisc + 4);   // [3 RC_MMAX]: sum x, sum y, count (8-aligned)
    const uint32_t tid = threadIdx.x, lane = lane_id(), wv = threadIdx.x >> 6;
    rt_binomials(L.bin);
    __syncthreads();
    for (uint32_t o = blockIdx.x; o < num_orders; o += gridDim.x) {
        const uint32_t a = off[o], n = off[o + 1] - a;
        if (n == 0) {
            if (tid == 0) {
                len_out[o] = 0;
                m_out[o] = 0;
            }
            continue;
        }
        const uint32_t *Dg = dist + mbase[o];
        for (uint32_t q = tid; q < n * n; q += blockDim.x) sF[q] = Dg[q];
        for (uint32_t q = tid; q < 2 * n; q += blockDim.x) sXY[q] = xy[2 * static_cast<size_t>(a) + q];
        __syncthreads();
        // ---- K-means (wave 0, lane = pick), growing m while a cluster is too big
        if (wv == 0) {
            const bool on = lane < n;
            const int64_t px = on ? sXY[2 * lane] : 0, py = on ? sXY[2 * lane + 1] : 0;
            bool bad = on && (px <= -65536 || px >= 65536 || py <= -65536 || py >= 65536);
            if (__builtin_amdgcn_ballot_w64(bad) != 0) {
                if (lane == 0) {
                    atomicOr(err, RC_ERR_RANGE);
                    sMisc[1] = 0xFFFFFFFFu;
                }
            } else {
                uint32_t mm = m0, used = 0xFFFFFFFFu;
                for (; mm <= RC_MMAX; ++mm) {
                    const uint32_t asg = wave_kmeans(on, px, py, n, mm, sXY, sCen, sAsg);
                    // cluster sizes
                    uint32_t big = 0;
                    for (uint32_t c = 0; c < mm && c < n; ++c) {
                        const uint32_t sz = static_cast<uint32_t>(
                            __builtin_popcountll(__builtin_amdgcn_ballot_w64(on && asg == c)));
                        if (sz > RT_NMAX) big = 1;
                    }
                    if (!big) {
                        used = mm;
                        break;
                    }
                }
                if (lane == 0) {
                    if (used == 0xFFFFFFFFu) atomicOr(err, RC_ERR_CLUSTER);
                    sMisc[0] = used;
                    sMisc[1] = used == 0xFFFFFFFFu ? 0xFFFFFFFFu : 0u;
                }
            }
        }
        __syncthreads();
        if (sMisc[1] == 0xFFFFFFFFu) {   // this order cannot be served; the call fails
            if (tid == 0) {
                len_out[o] = ~0ull;
                m_out[o] = 0;
            }
            __syncthreads();
            continue;
        }
        // ---- each non-empty cluster: its picks in index order, their route
        const uint32_t mm = sMisc[0];
        uint32_t ncl = 0, pos = 0;
        bool ovf = false;
        for (uint32_t c = 0; c < mm; ++c) {
            uint32_t k = 0;
            for (uint32_t i = 0; i < n; ++i) k += sAsg[i] == c;   // uniform: every thread counts
            if (k == 0) continue;
            if (tid == 0) {
                uint32_t w = 0;
                for (uint32_t i = 0; i < n; ++i)
                    if (sAsg[i] == c) sRoute[pos + w++] = i;   // members, index order
            }
            __syncthreads();
            for (uint32_t q = tid; q < k * k; q += blockDim.x)
                L.D[q] = sF[sRoute[pos + q / k] * n + sRoute[pos + q % k]];
            __syncthreads();
            rt_tables(L, k);   // the chaining below rebuilds them for the clusters
            rt_solve(L, k, ovf);
            if (tid == 0) {
                uint32_t loc[RT_NMAX], mem[RT_NMAX];
                rt_read_route(L, k, loc);
                for (uint32_t t = 0; t < k; ++t) mem[t] = sRoute[pos + t];
                for (uint32_t t = 0; t < k; ++t) sRoute[pos + t] = mem[loc[t]];
                uint32_t fl = 0, rl = 0;
                bool dummy = false;
                for (uint32_t t = 0; t + 1 < k; ++t) {
                    fl = rt_step(fl, sF[sRoute[pos + t] * n + sRoute[pos + t + 1]], ovf);
                    rl = rt_step(rl, sF[sRoute[pos + t + 1] * n + sRoute[pos + t]], ovf);
                }
                (void)dummy;
                sCl[4 * ncl] = pos;
                sCl[4 * ncl + 1] = k;
                sCl[4 * ncl + 2] = fl;
                sCl[4 * ncl + 3] = rl;
            }
            __syncthreads();
            ++ncl;
            pos += k;
        }
        // ---- chaining: subset programme over the ncl clusters (pieces (c, o))
        rt_tables(L, ncl);
        uint32_t *G = L.H;   // state (S, c, o) at (base[S] + rank of c in S) * 2 + o
        {
            constexpr uint32_t NB1 = RT_NMAX + 1;
            for (uint32_t q = tid; q < 2 * ncl; q += blockDim.x) {
                const uint32_t c = q >> 1, o = q & 1u;
                G[L.base[1u << c] * 2 + o] = sCl[4 * c + 2 + o];
            }
            __syncthreads();
            uint32_t lstart = 1 + ncl;
            for (uint32_t k = 2; k <= ncl; ++k) {
                const uint32_t items = L.bin[ncl * NB1 + k] * k;
                for (uint32_t q = tid; q < items; q += blockDim.x) {
                    const uint32_t r = q / k, mi = q - r * k;
                    const uint32_t S = L.ord[lstart + r];
                    uint32_t T = S;
                    for (uint32_t x = 0; x < mi; ++x) T &= T - 1u;
                    const uint32_t c = __builtin_ctz(T);
                    const uint32_t R = S & ~(1u << c);
                    const uint32_t bR = L.base[R];
                    for (uint32_t o = 0; o < 2; ++o) {
                        const uint32_t p0 = sCl[4 * c], k0 = sCl[4 * c + 1];
                        const uint32_t end = o ? sRoute[p0] : sRoute[p0 + k0 - 1];
                        uint32_t inner = INF, rj = 0;
                        for (uint32_t U = R; U != 0; U &= U - 1u, ++rj) {
                            const uint32_t c2 = __builtin_ctz(U);
                            const uint32_t p2 = sCl[4 * c2], k2 = sCl[4 * c2 + 1];
                            inner = min(inner, rt_step(G[(bR + rj) * 2], sF[end * n + sRoute[p2]], ovf));
                            inner = min(inner, rt_step(G[(bR + rj) * 2 + 1], sF[end * n + sRoute[p2 + k2 - 1]], ovf));
                        }
                        G[(L.base[S] + mi) * 2 + o] = rt_step(inner, sCl[4 * c + 2 + o], ovf);
                    }
                }
                lstart += L.bin[ncl * NB1 + k];
                __syncthreads();
            }
        }
        if (ovf) atomicOr(err, RC_ERR_RANGE);
        if (tid == 0) {
            // the cheapest first piece, then greedily the smallest next piece
            const uint32_t all = (1u << ncl) - 1u, bA = L.base[all];
            uint32_t best = INF;
            for (uint32_t x = 0; x < 2 * ncl; ++x) best = min(best, G[bA * 2 + x]);
            uint32_t x = 0;
            while (G[bA * 2 + x] != best) ++x;
            uint32_t cc = x >> 1, oo = x & 1u, S = all, w = 0;
            bool dummy = false;
            for (;;) {
                const uint32_t p0 = sCl[4 * cc], k0 = sCl[4 * cc + 1];
                for (uint32_t t = 0; t < k0; ++t) route_out[a + w++] = oo ? sRoute[p0 + k0 - 1 - t] : sRoute[p0 + t];
                const uint32_t R = S & ~(1u << cc);
                if (!R) break;
                const uint32_t bR = L.base[R], end = oo ? sRoute[p0] : sRoute[p0 + k0 - 1];
                uint32_t inner = INF, rj = 0;
                for (uint32_t U = R; U != 0; U &= U - 1u, ++rj) {
                    const uint32_t c2 = __builtin_ctz(U);
                    const uint32_t p2 = sCl[4 * c2], k2 = sCl[4 * c2 + 1];
                    inner = min(inner, rt_step(G[(bR + rj) * 2], sF[end * n + sRoute[p2]], dummy));
                    inner = min(inner, rt_step(G[(bR + rj) * 2 + 1], sF[end * n + sRoute[p2 + k2 - 1]], dummy));
                }
                uint32_t nc = 0, no = 0;
                rj = 0;
                for (uint32_t U = R; U != 0; U &= U - 1u, ++rj) {
                    const uint32_t c2 = __builtin_ctz(U);
                    const uint32_t p2 = sCl[4 * c2], k2 = sCl[4 * c2 + 1];
                    if (rt_step(G[(bR + rj) * 2], sF[end * n + sRoute[p2]], dummy) == inner) {
                        nc = c2;
                        no = 0;
                        break;
                    }
                    if (rt_step(G[(bR + rj) * 2 + 1], sF[end * n + sRoute[p2 + k2 - 1]], dummy) == inner) {
                        nc = c2;
                        no = 1;
                        break;
                    }
                }
                S = R;
                cc = nc;
                oo = no;
            }
            len_out[o] = best == INF ? ~0ull : static_cast<uint64_t>(best);
            m_out[o] = mm;
        }
        __syncthreads();   // the next order reuses the LDS
    }
}

// The paper's route-permutation structure (numerical experiments, the
// CUDA kernel that evaluates every ordering in its own thread), kept as the
// baseline of the subset programme: thread q of order o takes the q-th
// ordering in lexicographic order (factorial-base digits pick the q-th
// unused stop at each position), sums its n-1 steps in 32 bits with WR_INF
// absorbing, and the order's minimum of (length << 22 | q) is kept with a
// 64-bit atomic minimum; the smallest rank among the shortest orderings is
// the lexicographically smallest one, as the subset programme returns.
constexpr uint32_t RP_NMAX = 10;   // 10! = 3,628,800 < 2^22 orderings
__global__ __launch_bounds__(256) void k_route_perm(uint32_t num_orders, const uint32_t *__restrict__ off,
                                                    const uint64_t *__restrict__ mbase,
                                                    const uint32_t *__restrict__ dist,
                                                    unsigned long long *__restrict__ best,
                                                    uint32_t *__restrict__ overflow) {
    __shared__ unsigned long long s_best[256];
    for (uint32_t o = blockIdx.y; o < num_orders; o += gridDim.y) {
        const uint32_t a = off[o], n = off[o + 1] - a;
        uint32_t fact = 1;
        for (uint32_t x = 2; x <= n; ++x) fact *= x;
        const uint32_t *D = dist + mbase[o];
        unsigned long long mine = ~0ull;
        bool ovf = false;
        for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; n > 0 && q < fact; q += gridDim.x * blockDim.x) {
            uint32_t r = q, f = fact, used = 0, prev = 0, len = 0;
            for (uint32_t x = 0; x < n; ++x) {
                f /= (n - x);
                uint32_t d = r / f;
                r -= d * f;
                uint32_t c = 0;
                for (;; ++c)
                    if (!((used >> c) & 1u) && d-- == 0) break;
                used |= 1u << c;
                if (x > 0) len = rt_step(len, D[prev * n + c], ovf);
                prev = c;
            }
            const unsigned long long key = (static_cast<unsigned long long>(len) << 22) | q;
            mine = key < mine ? key : mine;
        }
        if (ovf) atomicOr(overflow, 1u);
        s_best[threadIdx.x] = mine;
        __syncthreads();
        for (uint32_t h = blockDim.x >> 1; h > 0; h >>= 1) {
            if (threadIdx.x < h && s_best[threadIdx.x + h] < s_best[threadIdx.x]) s_best[threadIdx.x] = s_best[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0 && n > 0) atomicMin(best + o, s_best[0]);
        __syncthreads();
    }
}

// Orderings and lengths from the per-order keys of k_route_perm.
__global__ void k_route_perm_out(uint32_t num_orders, const uint32_t *__restrict__ off,
                                 const unsigned long long *__restrict__ best, uint64_t *__restrict__ len_out,
                                 uint32_t *__restrict__ route_out) {
    for (uint32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < num_orders; o += gridDim.x * blockDim.x) {
        const uint32_t a = off[o], n = off[o + 1] - a;
        if (n == 0) {
            len_out[o] = 0;
            continue;
        }
        const unsigned long long key = best[o];
        const uint32_t len = static_cast<uint32_t>(key >> 22);
        uint32_t r = static_cast<uint32_t>(key & ((1u << 22) - 1u)), f = 1, used = 0;
        for (uint32_t x = 2; x <= n; ++x) f *= x;
        for (uint32_t x = 0; x < n; ++x) {
            f /= (n - x);
            uint32_t d = r / f;
            r -= d * f;
            uint32_t c = 0;
            for (;; ++c)
                if (!((used >> c) & 1u) && d-- == 0) break;
            used |= 1u << c;
            route_out[a + x] = c;
        }
        len_out[o] = len == INF ? ~0ull : static_cast<uint64_t>(len);
    }
}

uint32_t route_enumerate_max_stops() { return RP_NMAX; }

void launch_route_perm(uint32_t num_orders, const uint32_t *off, const uint64_t *mbase, const uint32_t *dist,
                       unsigned long long *best, uint64_t *len_out, uint32_t *route_out, uint32_t *overflow,
                       uint32_t nmax, hipStream_t st) {
    if (!num_orders) return;
    uint32_t fact = 1;
    for (uint32_t x = 2; x <= nmax; ++x) fact *= x;
    dim3 grid(std::max(1u, std::min(1024u, (fact + 255) / 256)), std::min(num_orders, 65535u));
    hipLaunchKernelGGL(k_route_perm, grid, 256, 0, st, num_orders, off, mbase, dist, best, overflow);
    check_launch("route_perm");
    hipLaunchKernelGGL(k_route_perm_out, blocks_for(num_orders, 256, 1024), 256, 0, st, num_orders, off, best,
                       len_out, route_out);
    check_launch("route_perm_out");
}

uint32_t route_max_stops() { return RT_NMAX; }

uint32_t route_lds_bytes(uint32_t nmax) { return rt_lds_words(nmax) * 4u; }

uint32_t route_clustered_lds_bytes() {
    return (rt_lds_words(RT_NMAX) + RC_NMAX * RC_NMAX + 2 * RC_NMAX + 2 * RC_NMAX + 4 * RC_MMAX + 4 +
            2 * 3 * RC_MMAX) * 4u;
}
uint32_t route_clustered_max_stops() { return RC_NMAX; }
uint32_t route_clustered_max_clusters() { return RC_MMAX; }

void launch_route_clustered(uint32_t num_orders, const uint32_t *off, const uint64_t *mbase, const uint32_t *dist,
                            const int32_t *xy, uint32_t m, uint64_t *len_out, uint32_t *route_out, uint32_t *m_out,
                            uint32_t *err, uint32_t grid, hipStream_t st) {
    if (!num_orders) return;
    hipLaunchKernelGGL(k_route_clustered, std::min(grid, num_orders), RT_THREADS, route_clustered_lds_bytes(), st,
                       num_orders, off, mbase, dist, xy, m, len_out, route_out, m_out, err);
    check_launch("route_clustered");
}

void launch_route_hk(uint32_t num_orders, const uint32_t *off, const uint64_t *mbase, const uint32_t *dist,
                     uint64_t *len_out, uint32_t *route_out, uint32_t *overflow, uint32_t nmax, uint32_t grid,
                     hipStream_t st) {
    if (!num_orders) return;
    const uint32_t n = std::max(nmax, 1u);
    hipLaunchKernelGGL(k_route_hk, std::min(grid, num_orders), RT_THREADS, route_lds_bytes(n), st, num_orders,
                       off, mbase, dist, len_out, route_out, overflow, n);
    check_launch("route_hk");
}

}  // namespace wr
