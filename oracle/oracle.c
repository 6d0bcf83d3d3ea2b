/*
 * Reference oracle for the warehouse routing hot path -- TEST INFRASTRUCTURE.
 *
 * Plain, slow, obviously-correct CPU code.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may call it; the product path
 * never links or loads it, and it shares no source, header or helper with the
 * HIP library.
 *
 * What it computes is the plain definition of the result the paper's routing
 * step reaches: for a directed graph with non-negative integer arc weights,
 * d(s, v) = minimum over s->v paths of the sum of arc weights, INF if no path
 * exists (GPU implementation subsection: Bellman-Ford over integer edge
 * arrays, validated against Dijkstra on the CPU, which the closing remark of
 * that subsection says gave identical shortest paths).  Two independent
 * algorithms reach that definition here:
 *
 *   - Dijkstra with a binary heap and lazy deletion (64-bit accumulation);
 *   - Jacobi Bellman-Ford: d_0 = INF except d_0(s) = 0, then
 *     d_{k+1}(v) = min(d_k(v), min_{(u,v)} d_k(u) + w(u,v)), stopping when a
 *     round changes nothing or after V-1 rounds (the round count the paper
 *     runs).
 *
 * plus the canonical predecessor (smallest tight in-neighbour id), the
 * per-order pick-to-pick matrices D_o[i][j] = d(p_i, p_j) (routes are built
 * over stop-to-stop distances, Route Optimization section), CSR validation
 * with the overflow bound, and a certificate checker that proves a
 * (dist, pred) pair optimal without re-solving.
 *
 * Conventions: INF = 0xFFFFFFFF, "no predecessor" = -1, vertex ids < 2^31.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_INF 0xFFFFFFFFu

/* ------------------------------------------------------------------ */
/* validation                                                          */
/* ------------------------------------------------------------------ */

/* 0 = ok, 1 = malformed CSR, 2 = a shortest path could reach INF.
 * Rules: row_ptr[0] = 0, row_ptr non-decreasing, row_ptr[V] = E, every
 * col < V.  Overflow bound: max_w * (number of vertices incident to an arc
 * minus 1) must stay below INF, since a simple path visits each such vertex
 * at most once. */
int orc_validate_csr(uint32_t V, uint32_t E, const uint32_t *row_ptr,
                     const uint32_t *col, const uint32_t *w)
{
    if (V == 0 || V >= 0x80000000u || !row_ptr) return 1;
    if (E > 0 && (!col || !w)) return 1;
    if (row_ptr[0] != 0 || row_ptr[V] != E) return 1;
    for (uint32_t v = 0; v < V; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return 1;
    for (uint32_t e = 0; e < E; ++e)
        if (col[e] >= V) return 1;
    unsigned char *inc = (unsigned char *)calloc(V, 1);
    if (!inc) return 1;
    uint64_t maxw = 0, n_inc = 0;
    for (uint32_t u = 0; u < V; ++u)
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            inc[u] = 1;
            inc[col[e]] = 1;
            if (w[e] > maxw) maxw = w[e];
        }
    for (uint32_t v = 0; v < V; ++v) n_inc += inc[v];
    free(inc);
    if (n_inc > 1 && maxw * (n_inc - 1) >= (uint64_t)ORC_INF) return 2;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dijkstra                                                            */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t key; uint32_t v; } heap_item;

static void heap_push(heap_item *h, size_t *n, heap_item it)
{
    size_t i = (*n)++;
    while (i > 0) {
        size_t p = (i - 1) / 2;
        if (h[p].key <= it.key) break;
        h[i] = h[p];
        i = p;
    }
    h[i] = it;
}

static heap_item heap_pop(heap_item *h, size_t *n)
{
    heap_item top = h[0];
    heap_item last = h[--(*n)];
    size_t i = 0;
    for (;;) {
        size_t l = 2 * i + 1, r = l + 1, m = i;
        uint64_t mk = last.key;
        if (l < *n && h[l].key < mk) { m = l; mk = h[l].key; }
        if (r < *n && h[r].key < mk) { m = r; }
        if (m == i) break;
        h[i] = h[m];
        i = m;
    }
    if (*n > 0) h[i] = last;
    return top;
}

/* Single-source Dijkstra; dist must hold V entries.  0 = ok, 3 = no memory. */
int orc_dijkstra(uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                 const uint32_t *w, uint32_t src, uint32_t *dist)
{
    uint32_t E = row_ptr[V];
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * V);
    unsigned char *done = (unsigned char *)calloc(V, 1);
    heap_item *h = (heap_item *)malloc(sizeof(heap_item) * ((size_t)E + 1));
    if (!d || !done || !h) { free(d); free(done); free(h); return 3; }
    for (uint32_t v = 0; v < V; ++v) d[v] = UINT64_MAX;
    size_t n = 0;
    d[src] = 0;
    heap_item s0 = {0, src};
    heap_push(h, &n, s0);
    while (n > 0) {
        heap_item it = heap_pop(h, &n);
        uint32_t u = it.v;
        if (done[u] || it.key != d[u]) continue;   /* stale entry */
        done[u] = 1;
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint32_t x = col[e];
            uint64_t nd = d[u] + (uint64_t)w[e];
            if (nd < d[x]) {
                d[x] = nd;
                heap_item ni = {nd, x};
                heap_push(h, &n, ni);
            }
        }
    }
    for (uint32_t v = 0; v < V; ++v)
        dist[v] = (d[v] >= (uint64_t)ORC_INF) ? ORC_INF : (uint32_t)d[v];
    free(d); free(done); free(h);
    return 0;
}

/* Dijkstra from each of S sources into dist[S*V] (source-major), in
 * parallel over sources on `nthreads` threads (0 = all).  Returns 0 or the
 * first error. */
int orc_dijkstra_multi(uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                       const uint32_t *w, uint32_t S, const uint32_t *sources,
                       uint32_t *dist, int nthreads)
{
    int err = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : err)
#endif
    for (long i = 0; i < (long)S; ++i)
        err |= orc_dijkstra(V, row_ptr, col, w, sources[i], dist + (size_t)i * V);
    (void)nthreads;
    return err;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Jacobi Bellman-Ford                                                 */
/* ------------------------------------------------------------------ */

/* Rounds of d_{k+1}(v) = min(d_k(v), min over arcs (u,v) of d_k(u)+w) until
 * a round changes nothing or `max_rounds` rounds ran (0 means V-1).
 * *rounds_out receives the number of rounds that changed something.
 * Returns 0, or 4 if the cap was hit while values were still changing. */
int orc_bellman_ford(uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                     const uint32_t *w, uint32_t src, uint32_t *dist,
                     uint32_t max_rounds, uint32_t *rounds_out)
{
    if (max_rounds == 0) max_rounds = V > 1 ? V - 1 : 1;
    uint64_t *cur = (uint64_t *)malloc(sizeof(uint64_t) * V);
    uint64_t *nxt = (uint64_t *)malloc(sizeof(uint64_t) * V);
    if (!cur || !nxt) { free(cur); free(nxt); return 3; }
    for (uint32_t v = 0; v < V; ++v) cur[v] = UINT64_MAX;
    cur[src] = 0;
    uint32_t rounds = 0;
    int changed = 1;
    while (changed && rounds < max_rounds) {
        changed = 0;
        memcpy(nxt, cur, sizeof(uint64_t) * V);
        for (uint32_t u = 0; u < V; ++u) {
            if (cur[u] == UINT64_MAX) continue;
            for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                uint64_t cand = cur[u] + (uint64_t)w[e];
                if (cand < nxt[col[e]]) nxt[col[e]] = cand;
            }
        }
        for (uint32_t v = 0; v < V; ++v)
            if (nxt[v] != cur[v]) { changed = 1; break; }
        uint64_t *t = cur; cur = nxt; nxt = t;
        if (changed) ++rounds;
    }
    /* one more check round tells whether the cap stopped a changing run */
    int capped = 0;
    if (changed) {
        for (uint32_t u = 0; u < V && !capped; ++u) {
            if (cur[u] == UINT64_MAX) continue;
            for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                if (cur[u] + (uint64_t)w[e] < cur[col[e]]) { capped = 1; break; }
        }
    }
    for (uint32_t v = 0; v < V; ++v)
        dist[v] = (cur[v] >= (uint64_t)ORC_INF) ? ORC_INF : (uint32_t)cur[v];
    if (rounds_out) *rounds_out = rounds;
    free(cur); free(nxt);
    return capped ? 4 : 0;
}

/* ------------------------------------------------------------------ */
/* canonical predecessor                                               */
/* ------------------------------------------------------------------ */

/* pred[v] = smallest u with an arc (u, v), d(u) != INF and
 * d(u) + w(u, v) = d(v); pred[src] = -1; unreachable vertices get -1. */
void orc_canonical_pred(uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                        const uint32_t *w, uint32_t src, const uint32_t *dist,
                        int32_t *pred)
{
    for (uint32_t v = 0; v < V; ++v) pred[v] = -1;
    for (uint32_t u = 0; u < V; ++u) {
        if (dist[u] == ORC_INF) continue;
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint32_t x = col[e];
            if (x == src || dist[x] == ORC_INF) continue;
            if ((uint64_t)dist[u] + w[e] == (uint64_t)dist[x])
                if (pred[x] < 0 || (uint32_t)pred[x] > u) pred[x] = (int32_t)u;
        }
    }
}

/* ------------------------------------------------------------------ */
/* order matrices                                                      */
/* ------------------------------------------------------------------ */

/* out receives, for every order o with picks p_0..p_{P-1}, the P x P block
 * D_o[i][j] = d(p_i, p_j) (row = source pick), blocks concatenated in order.
 * `dist_rows` maps each pick position k (0..total picks-1) to a row of
 * source-major distances already computed for vertex picks[k]. */
void orc_gather_orders(uint32_t V, uint32_t num_orders, const uint32_t *pick_off,
                       const uint32_t *picks, const uint32_t *row_of_pick,
                       const uint32_t *dist_rows, uint32_t *out)
{
    size_t o_base = 0;
    for (uint32_t o = 0; o < num_orders; ++o) {
        uint32_t a = pick_off[o], P = pick_off[o + 1] - a;
        for (uint32_t i = 0; i < P; ++i) {
            const uint32_t *row = dist_rows + (size_t)row_of_pick[a + i] * V;
            for (uint32_t j = 0; j < P; ++j)
                out[o_base + (size_t)i * P + j] = row[picks[a + j]];
        }
        o_base += (size_t)P * P;
    }
}

/* ------------------------------------------------------------------ */
/* certificate                                                         */
/* ------------------------------------------------------------------ */

/* Proves that dist (and pred, if not NULL) is a shortest-path solution from
 * src without re-solving.  Returns 0 if valid, else a code naming the first
 * failed condition:
 *   10 d(src) != 0
 *   11 an arc (u,v) with d(u) finite and d(v) > d(u) + w (infeasible)
 *   12 a finite d(v) not reachable from src through tight arcs
 *      (d(u) + w = d(v)), so d(v) is not the length of any path
 *   13 an INF vertex reachable from src
 *   20 pred[src] != -1, 21 pred set on an INF vertex or missing on a finite
 *      one, 22 pred[v] -> v is not a tight arc, 23 pred chain does not reach
 *      src (cycle)
 * Feasibility gives d(v) <= length of every s->v path; tight reachability
 * gives a path of length exactly d(v); together they prove optimality. */
int orc_certificate(uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                    const uint32_t *w, uint32_t src, const uint32_t *dist,
                    const int32_t *pred)
{
    if (dist[src] != 0) return 10;
    for (uint32_t u = 0; u < V; ++u) {
        if (dist[u] == ORC_INF) continue;
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if ((uint64_t)dist[col[e]] > (uint64_t)dist[u] + w[e]) return 11;
    }
    uint32_t *stack = (uint32_t *)malloc(sizeof(uint32_t) * V);
    unsigned char *seen = (unsigned char *)calloc(V, 1);
    unsigned char *reach = (unsigned char *)calloc(V, 1);
    if (!stack || !seen || !reach) { free(stack); free(seen); free(reach); return 3; }
    int rc = 0;
    /* tight-arc reachability */
    size_t n = 0;
    stack[n++] = src; seen[src] = 1;
    while (n) {
        uint32_t u = stack[--n];
        for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            uint32_t x = col[e];
            if (!seen[x] && (uint64_t)dist[u] + w[e] == (uint64_t)dist[x]) {
                seen[x] = 1; stack[n++] = x;
            }
        }
    }
    for (uint32_t v = 0; v < V && !rc; ++v)
        if (dist[v] != ORC_INF && !seen[v]) rc = 12;
    /* plain reachability */
    if (!rc) {
        n = 0; stack[n++] = src; reach[src] = 1;
        while (n) {
            uint32_t u = stack[--n];
            for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                if (!reach[col[e]]) { reach[col[e]] = 1; stack[n++] = col[e]; }
        }
        for (uint32_t v = 0; v < V && !rc; ++v)
            if (dist[v] == ORC_INF && reach[v]) rc = 13;
    }
    if (!rc && pred) {
        if (pred[src] != -1) rc = 20;
        for (uint32_t v = 0; v < V && !rc; ++v) {
            if (v == src) continue;
            if ((dist[v] == ORC_INF) != (pred[v] < 0)) { rc = 21; break; }
            if (pred[v] < 0) continue;
            uint32_t u = (uint32_t)pred[v];
            int tight = 0;
            if (u < V && dist[u] != ORC_INF)
                for (uint32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
                    if (col[e] == v && (uint64_t)dist[u] + w[e] == (uint64_t)dist[v]) { tight = 1; break; }
            if (!tight) rc = 22;
        }
        /* every chain must reach src: resolve depths iteratively */
        if (!rc) {
            memset(seen, 0, V);          /* 0 unknown, 1 on current chain, 2 ok */
            seen[src] = 2;
            for (uint32_t v = 0; v < V && !rc; ++v) {
                if (dist[v] == ORC_INF || seen[v] == 2) continue;
                n = 0;
                uint32_t x = v;
                while (seen[x] == 0) { seen[x] = 1; stack[n++] = x; x = (uint32_t)pred[x]; }
                if (seen[x] == 1) { rc = 23; break; }
                while (n) seen[stack[--n]] = 2;
            }
        }
    }
    free(stack); free(seen); free(reach);
    return rc;
}

/* orc_certificate of S source-major rows dist[S*V] (and pred[S*V] when
 * not NULL), in parallel over sources on `nthreads` threads (0 = all).
 * rc[i] receives the code of row i; returns the number of rows whose code
 * is not 0. */
int orc_certificate_multi(uint32_t V, const uint32_t *row_ptr, const uint32_t *col,
                          const uint32_t *w, uint32_t S, const uint32_t *sources,
                          const uint32_t *dist, const int32_t *pred, int32_t *rc, int nthreads)
{
    int bad = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : bad)
#endif
    for (long i = 0; i < (long)S; ++i) {
        rc[i] = orc_certificate(V, row_ptr, col, w, sources[i], dist + (size_t)i * V,
                                pred ? pred + (size_t)i * V : NULL);
        bad += rc[i] != 0;
    }
    (void)nthreads;
    return bad;
}

/* ------------------------------------------------------------------ */
/* Optimal open route over an order's stops (Route Optimization section:
 * the entrance/exit is not part of the route, so a route is an ordering of
 * the n stops with any first and any last stop, and its length is the sum
 * of the n-1 stop-to-stop distances along it; the section counts n!/2
 * routes by identifying the two travel directions, which for a directed
 * matrix are kept apart here).  The result is the minimum over all n!
 * orderings; among orderings of that length the lexicographically smallest
 * index sequence is returned.  Lengths are exact 64-bit sums; an INF entry
 * makes every ordering that uses it infinite (ORC_ROUTE_INF).
 *
 * The minimum is reached with Held and Karp's dynamic programme over stop
 * subsets, which the section names as the exact alternative to enumerating
 * orderings: h(S, i) = shortest path that starts at stop i and visits exactly
 * the stops of S (i in S), h({i}, i) = 0, h(S, i) = min over j in S\{i} of
 * D[i][j] + h(S\{i}, j).  The optimum is min_i h(all, i), and the
 * lexicographically smallest optimal ordering is read greedily: the smallest
 * i with h(all, i) optimal, then repeatedly the smallest j whose step
 * D[i][j] + h(rest, j) equals h(current, i).  When every ordering is
 * infinite they all tie and the smallest, 0, 1, ..., n-1, is returned.     */
#define ORC_ROUTE_INF UINT64_MAX

static uint64_t route_add(uint64_t a, uint32_t d)
{
    if (a == ORC_ROUTE_INF || d == ORC_INF) return ORC_ROUTE_INF;
    return a + d;
}

/* n <= 20; D row-major n x n; route gets n indices.  Returns 0, or -1 when
 * n is out of range or memory is short. */
int orc_route_held_karp(uint32_t n, const uint32_t *D, uint64_t *cost, uint32_t *route)
{
    if (n == 0) {
        *cost = 0;
        return 0;
    }
    if (n > 20) return -1;
    const size_t nsub = (size_t)1 << n;
    uint64_t *h = (uint64_t *)malloc(nsub * n * sizeof(uint64_t));
    if (!h) return -1;
    for (size_t k = 0; k < nsub * n; ++k) h[k] = ORC_ROUTE_INF;
    for (uint32_t i = 0; i < n; ++i) h[((size_t)1 << i) * n + i] = 0;
    /* subsets in increasing numeric order: S \ {i} < S, so it is final */
    for (size_t S = 1; S < nsub; ++S) {
        if ((S & (S - 1)) == 0) continue;   /* singletons are set */
        for (uint32_t i = 0; i < n; ++i) {
            if (!(S & ((size_t)1 << i))) continue;
            const size_t R = S & ~((size_t)1 << i);
            uint64_t best = ORC_ROUTE_INF;
            for (uint32_t j = 0; j < n; ++j) {
                if (!(R & ((size_t)1 << j))) continue;
                const uint64_t v = route_add(h[R * n + j], D[(size_t)i * n + j]);
                if (v < best) best = v;
            }
            h[S * n + i] = best;
        }
    }
    const size_t all = nsub - 1;
    uint64_t opt = ORC_ROUTE_INF;
    for (uint32_t i = 0; i < n; ++i)
        if (h[all * n + i] < opt) opt = h[all * n + i];
    if (opt == ORC_ROUTE_INF) {
        /* every ordering infinite: they all tie, the smallest is 0, 1, ... */
        for (uint32_t k = 0; k < n; ++k) route[k] = k;
        *cost = opt;
        free(h);
        return 0;
    }
    uint32_t cur = 0;
    while (h[all * n + cur] != opt) ++cur;
    size_t S = all;
    route[0] = cur;
    for (uint32_t k = 1; k < n; ++k) {
        const size_t R = S & ~((size_t)1 << cur);
        uint32_t nxt = 0;
        for (uint32_t j = 0; j < n; ++j) {
            if (!(R & ((size_t)1 << j))) continue;
            if (route_add(h[R * n + j], D[(size_t)cur * n + j]) == h[S * n + cur]) {
                nxt = j;
                break;
            }
        }
        route[k] = nxt;
        S = R;
        cur = nxt;
    }
    *cost = opt;
    free(h);
    return 0;
}

/* Every order of a batch: matrices concatenated (order o is P_o x P_o at the
 * running offset sum of P^2), routes concatenated at pick_off[o]. */
int orc_order_routes(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *D, uint64_t *cost,
                     uint32_t *route, int nthreads)
{
    uint64_t *base = (uint64_t *)malloc(((size_t)num_orders + 1) * sizeof(uint64_t));
    if (!base) return -1;
    base[0] = 0;
    for (uint32_t o = 0; o < num_orders; ++o) {
        const uint64_t P = pick_off[o + 1] - pick_off[o];
        base[o + 1] = base[o] + P * P;
    }
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
#endif
    for (int64_t o = 0; o < (int64_t)num_orders; ++o) {
        const uint32_t P = pick_off[o + 1] - pick_off[o];
        if (orc_route_held_karp(P, D + base[o], cost + o, route + pick_off[o]) != 0) bad |= 1;
    }
    free(base);
    return bad ? -1 : 0;
}

/* The optimal open route by its plain definition: every ordering of the n
 * stops (n <= 12), generated depth first with the smallest unused stop
 * first, i.e. in lexicographic order; a length is the sum of the ordering's
 * n-1 steps (ORC_ROUTE_INF once a step is INF).  The first ordering of the
 * smallest length is kept: the lexicographically smallest of the shortest.
 * *count = orderings compared (n!).  A second, independent method beside
 * the subset programme above.  Returns 0, or -1 for n > 12. */
int orc_route_enumerate(uint32_t n, const uint32_t *D, uint64_t *cost, uint32_t *route, uint64_t *count)
{
    if (n > 12) return -1;
    *count = 1;
    *cost = 0;
    if (n <= 1) {
        if (n == 1) route[0] = 0;
        return 0;
    }
    uint32_t cur[12], used = 0;
    uint64_t part[12];
    int d = 0, have = 0;
    *count = 0;
    cur[0] = 0;
    for (;;) {
        while (cur[d] < n && (used & (1u << cur[d]))) ++cur[d];
        if (cur[d] >= n) {
            if (d == 0) break;
            --d;
            used &= ~(1u << cur[d]);
            ++cur[d];
            continue;
        }
        part[d] = d == 0 ? 0 : route_add(part[d - 1], D[(size_t)cur[d - 1] * n + cur[d]]);
        if ((uint32_t)d + 1 == n) {
            ++*count;
            if (!have || part[d] < *cost) {
                have = 1;
                *cost = part[d];
                for (uint32_t k = 0; k < n; ++k) route[k] = cur[k];
            }
            ++cur[d];
            continue;
        }
        used |= 1u << cur[d];
        ++d;
        cur[d] = 0;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Cluster-decomposed route (Route Optimization section, the theorem on
 * m clusters): the order's stops are split into m clusters by K-means on
 * their positions (clusters of an order, routes-and-clusters subsection;
 * a cluster's centre is the mean position of its picks, so a stop picked
 * twice weighs twice), an optimal open route is found inside every cluster,
 * and the global route is the cheapest way to chain the cluster routes:
 * every order of the clusters and every orientation of each cluster's
 * route, adding the steps between consecutive clusters' ends.
 *
 * Readings where the section is silent (the product library follows the
 * same ones):
 *  - positions are integer (x, y) pairs; squared Euclidean distances to a
 *    centre sum/c are compared exactly as |c*p - sum|^2 scaled by the other
 *    cluster's c^2 (64-bit integers);
 *  - initial centres by farthest-point selection: the first pick, then
 *    repeatedly the pick farthest (squared distance) from every chosen
 *    centre, ties to the smaller index; Lloyd iterations assign each pick
 *    to its nearest centre (ties to the smaller cluster index) and move
 *    every non-empty cluster's centre to its mean, until no assignment
 *    changes or 100 iterations;
 *  - a cluster's route is the optimal directed open route of orc_route_
 *    held_karp over its picks in increasing index order; a reversed cluster
 *    route costs its reversed steps;
 *  - chaining: non-empty clusters are numbered in cluster index order; the
 *    cheapest chain over every order and orientation of their routes is
 *    found by a subset programme, and among the cheapest the
 *    lexicographically smallest sequence of (cluster, orientation) is
 *    returned (forward before reversed);
 *  - if K-means leaves a cluster with more than max_cluster picks, m grows
 *    by one and the clustering restarts (up to m_max).
 * Lengths are exact 64-bit sums with ORC_ROUTE_INF absorbing.             */
static int64_t km_cmp(int64_t px, int64_t py, int64_t sxa, int64_t sya, int64_t ca, int64_t sxb, int64_t syb,
                      int64_t cb)
{
    /* sign of |p - s_a/c_a|^2 - |p - s_b/c_b|^2 */
    const int64_t dxa = ca * px - sxa, dya = ca * py - sya;
    const int64_t dxb = cb * px - sxb, dyb = cb * py - syb;
    const __int128 a = (__int128)(dxa * dxa + dya * dya) * (cb * cb);
    const __int128 b = (__int128)(dxb * dxb + dyb * dyb) * (ca * ca);
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* K-means of n points into m clusters; asg[i] = cluster of point i */
void orc_kmeans(uint32_t n, const int32_t *xy, uint32_t m, uint32_t *asg)
{
    int64_t sx[16], sy[16], cnt[16];
    uint32_t cen[16];
    uint32_t nc = 0;
    /* farthest-point initial centres (point indices) */
    cen[nc++] = 0;
    while (nc < m && nc < n) {
        int64_t best = -1;
        uint32_t bi = 0;
        for (uint32_t i = 0; i < n; ++i) {
            int64_t dmin = INT64_MAX;
            for (uint32_t c = 0; c < nc; ++c) {
                const int64_t dx = (int64_t)xy[2 * i] - xy[2 * cen[c]], dy = (int64_t)xy[2 * i + 1] - xy[2 * cen[c] + 1];
                const int64_t d = dx * dx + dy * dy;
                if (d < dmin) dmin = d;
            }
            if (dmin > best) {
                best = dmin;
                bi = i;
            }
        }
        cen[nc++] = bi;
    }
    for (uint32_t c = 0; c < nc; ++c) {
        sx[c] = xy[2 * cen[c]];
        sy[c] = xy[2 * cen[c] + 1];
        cnt[c] = 1;
    }
    for (uint32_t i = 0; i < n; ++i) asg[i] = 0xFFFFFFFFu;
    for (int it = 0; it < 100; ++it) {
        int changed = 0;
        for (uint32_t i = 0; i < n; ++i) {
            uint32_t b = 0;
            for (uint32_t c = 1; c < nc; ++c)
                if (km_cmp(xy[2 * i], xy[2 * i + 1], sx[c], sy[c], cnt[c], sx[b], sy[b], cnt[b]) < 0) b = c;
            if (asg[i] != b) {
                asg[i] = b;
                changed = 1;
            }
        }
        if (!changed) break;
        int64_t nsx[16] = {0}, nsy[16] = {0}, ncnt[16] = {0};
        for (uint32_t i = 0; i < n; ++i) {
            nsx[asg[i]] += xy[2 * i];
            nsy[asg[i]] += xy[2 * i + 1];
            ncnt[asg[i]] += 1;
        }
        for (uint32_t c = 0; c < nc; ++c)
            if (ncnt[c]) {
                sx[c] = nsx[c];
                sy[c] = nsy[c];
                cnt[c] = ncnt[c];
            }
    }
}

static uint64_t route_len(const uint32_t *D, uint32_t n, const uint32_t *r, uint32_t k, int reversed)
{
    uint64_t s = 0;
    for (uint32_t t = 0; t + 1 < k; ++t) {
        const uint32_t a = reversed ? r[k - 1 - t] : r[t], b = reversed ? r[k - 2 - t] : r[t + 1];
        s = route_add(s, D[(size_t)a * n + b]);
    }
    return s;
}

/* Length of a chain of cluster routes ("pieces"): piece c in orientation o
 * (0 forward, 1 reversed) starts at pstart[c][o], ends at pend[c][o] and
 * costs plen[c][o]; consecutive pieces are joined by the step from the end
 * of one to the start of the next. */
static uint64_t add64(uint64_t a, uint64_t b)
{
    if (a == ORC_ROUTE_INF || b == ORC_ROUTE_INF) return ORC_ROUTE_INF;
    return a + b;
}

struct chain_pieces {
    uint32_t K, n;
    const uint32_t *D;
    uint32_t pstart[16][2], pend[16][2];
    uint64_t plen[16][2];
};

/* The cheapest chain by its plain definition: every order of the K pieces
 * and every orientation of each.  Chains are generated depth first with the
 * smallest unused cluster first and forward before reversed, i.e. in
 * lexicographic order of their (cluster, orientation) sequences; the first
 * chain of the smallest length is kept, which is the lexicographically
 * smallest among the cheapest.  *count = chains compared (K! 2^K). */
static void chain_enumerate(const struct chain_pieces *P, uint64_t *best, uint32_t *bc, uint32_t *bo,
                            uint64_t *count)
{
    const uint32_t K = P->K;
    uint32_t sc[16], so[16];
    uint64_t part[16];
    uint32_t used = 0;
    int d = 0;
    *best = ORC_ROUTE_INF;
    *count = 0;
    int have = 0;
    /* the next candidate at depth d continues from (sc[d], so[d]) */
    sc[0] = 0;
    so[0] = 0;
    for (;;) {
        /* find the next unused (cluster, orientation) at depth d from sc/so */
        while (sc[d] < K && (used & (1u << sc[d]))) {
            ++sc[d];
            so[d] = 0;
        }
        if (sc[d] >= K) {
            if (d == 0) break;
            --d;
            used &= ~(1u << sc[d]);
            if (++so[d] == 2) {
                so[d] = 0;
                ++sc[d];
            }
            continue;
        }
        const uint32_t c = sc[d], o = so[d];
        part[d] = d == 0 ? P->plen[c][o]
                         : add64(add64(part[d - 1], route_add(0, P->D[(size_t)P->pend[sc[d - 1]][so[d - 1]] * P->n +
                                                                       P->pstart[c][o]])),
                                 P->plen[c][o]);
        if ((uint32_t)d + 1 == K) {
            ++*count;
            if (!have || part[d] < *best) {
                have = 1;
                *best = part[d];
                for (uint32_t k = 0; k < K; ++k) {
                    bc[k] = sc[k];
                    bo[k] = so[k];
                }
            }
            if (++so[d] == 2) {
                so[d] = 0;
                ++sc[d];
            }
            continue;
        }
        used |= 1u << c;
        ++d;
        sc[d] = 0;
        so[d] = 0;
    }
}

/* The same minimum by a subset programme (kept as a second method and
 * checked against the enumeration): g(S, c, o) is the cheapest chain that
 * starts with piece (c, o) and uses exactly the clusters of S, g({c}, c, o)
 * = len(c, o), g(S, c, o) = len(c, o) + min over c' in S\{c}, o' of the
 * step end(c, o) -> start(c', o') + g(S\{c}, c', o'); read back greedily
 * (smallest cluster, then orientation) it gives the same lexicographically
 * smallest cheapest chain. */
static int chain_subsets(const struct chain_pieces *P, uint64_t *best, uint32_t *bc, uint32_t *bo)
{
    const uint32_t K = P->K, nsK = 1u << K;
    uint64_t *gtab = (uint64_t *)malloc((size_t)nsK * K * 2 * sizeof(uint64_t));
    if (!gtab) return -1;
#define G(S_, c_, o_) gtab[((size_t)(S_) * K + (c_)) * 2 + (o_)]
#define STEP(c_, o_, c2_, o2_) route_add(0, P->D[(size_t)P->pend[c_][o_] * P->n + P->pstart[c2_][o2_]])
    for (uint32_t S = 1; S < nsK; ++S)
        for (uint32_t c = 0; c < K; ++c) {
            if (!(S & (1u << c))) continue;
            const uint32_t R = S & ~(1u << c);
            for (uint32_t o = 0; o < 2; ++o) {
                uint64_t inner = R ? ORC_ROUTE_INF : 0;
                for (uint32_t c2 = 0; c2 < K; ++c2) {
                    if (!(R & (1u << c2))) continue;
                    for (uint32_t o2 = 0; o2 < 2; ++o2) {
                        const uint64_t v = add64(G(R, c2, o2), STEP(c, o, c2, o2));
                        if (v < inner) inner = v;
                    }
                }
                G(S, c, o) = add64(inner, P->plen[c][o]);
            }
        }
    uint64_t opt = ORC_ROUTE_INF;
    for (uint32_t c = 0; c < K; ++c)
        for (uint32_t o = 0; o < 2; ++o)
            if (G(nsK - 1, c, o) < opt) opt = G(nsK - 1, c, o);
    /* every chain infinite: they all tie, the smallest sequence is every
     * cluster in index order, forward */
    if (opt == ORC_ROUTE_INF) {
        for (uint32_t k = 0; k < K; ++k) {
            bc[k] = k;
            bo[k] = 0;
        }
        free(gtab);
        *best = opt;
        return 0;
    }
    uint32_t cc = 0, oo = 0;
    while (G(nsK - 1, cc, oo) != opt) {
        if (++oo == 2) {
            oo = 0;
            ++cc;
        }
    }
    uint32_t S = nsK - 1;
    for (uint32_t k = 0;; ++k) {
        bc[k] = cc;
        bo[k] = oo;
        const uint32_t R = S & ~(1u << cc);
        if (!R) break;
        /* finite here: the rest of the chain must cost G(S, cc, oo) - len */
        const uint64_t want = G(S, cc, oo) - P->plen[cc][oo];
        uint32_t nc2 = 0, no2 = 0;
        int found = 0;
        for (uint32_t c2 = 0; c2 < K && !found; ++c2) {
            if (!(R & (1u << c2))) continue;
            for (uint32_t o2 = 0; o2 < 2 && !found; ++o2)
                if (add64(G(R, c2, o2), STEP(cc, oo, c2, o2)) == want) {
                    nc2 = c2;
                    no2 = o2;
                    found = 1;
                }
        }
        S = R;
        cc = nc2;
        oo = no2;
    }
#undef STEP
#undef G
    free(gtab);
    *best = opt;
    return 0;
}

/* Chains K <= 16 cluster routes (pieces) over an n x n matrix D: piece k
 * holds sizes[k] stop indices at stops + (sizes[0] + ... + sizes[k-1]);
 * writes the cheapest chain's stops into route (n entries), its length into
 * *cost and, with the enumeration, the chains compared into *count
 * (by_subsets != 0 uses the subset programme instead; *count is then 0).
 * Returns 0, or -1 for a bad size or short memory. */
int orc_chain_routes(uint32_t K, const uint32_t *sizes, const uint32_t *stops, uint32_t n, const uint32_t *D,
                     int by_subsets, uint64_t *cost, uint32_t *route, uint64_t *count)
{
    if (K == 0 || K > 16) return -1;
    struct chain_pieces P;
    P.K = K;
    P.n = n;
    P.D = D;
    const uint32_t *first[16];
    uint32_t at = 0;
    for (uint32_t c = 0; c < K; ++c) {
        if (sizes[c] == 0) return -1;
        first[c] = stops + at;
        at += sizes[c];
        const uint32_t k = sizes[c];
        P.pstart[c][0] = first[c][0];
        P.pend[c][0] = first[c][k - 1];
        P.pstart[c][1] = P.pend[c][0];
        P.pend[c][1] = P.pstart[c][0];
        P.plen[c][0] = route_len(D, n, first[c], k, 0);
        P.plen[c][1] = route_len(D, n, first[c], k, 1);
    }
    uint32_t bc[16], bo[16];
    uint64_t cnt = 0;
    if (by_subsets) {
        if (chain_subsets(&P, cost, bc, bo)) return -1;
    } else {
        chain_enumerate(&P, cost, bc, bo, &cnt);
    }
    if (count) *count = cnt;
    uint32_t w = 0;
    for (uint32_t k = 0; k < K; ++k) {
        const uint32_t c = bc[k], s = sizes[c];
        for (uint32_t t = 0; t < s; ++t) route[w++] = bo[k] ? first[c][s - 1 - t] : first[c][t];
    }
    return 0;
}

/* n <= 64 stops, positions xy[2n]; m clusters requested (1..16), clusters
 * of at most max_cluster (<= 20) stops, m grown up to m_max (<= 16).  Writes
 * the global route (indices 0..n-1) and its length; *m_used = clusters
 * used.  The clusters' routes are chained by enumeration.  Returns 0, or -1
 * when no m <= m_max keeps every cluster small. */
int orc_route_clustered(uint32_t n, const uint32_t *D, const int32_t *xy, uint32_t m, uint32_t max_cluster,
                        uint32_t m_max, uint64_t *cost, uint32_t *route, uint32_t *m_used)
{
    if (n == 0) {
        *cost = 0;
        *m_used = 0;
        return 0;
    }
    if (n > 64 || m == 0 || m_max > 16 || max_cluster > 20) return -1;
    uint32_t asg[64];
    uint32_t mm = m;
    for (;; ++mm) {
        if (mm > m_max) return -1;
        orc_kmeans(n, xy, mm, asg);
        uint32_t sz[16] = {0};
        for (uint32_t i = 0; i < n; ++i) sz[asg[i]]++;
        int ok = 1;
        for (uint32_t c = 0; c < mm; ++c)
            if (sz[c] > max_cluster) ok = 0;
        if (ok) break;
    }
    /* per non-empty cluster (in cluster index order): its picks in index
     * order and their optimal route */
    uint32_t sizes[16], stops[64], ncl = 0, at = 0;
    for (uint32_t c = 0; c < mm; ++c) {
        uint32_t members[64], k = 0;
        for (uint32_t i = 0; i < n; ++i)
            if (asg[i] == c) members[k++] = i;
        if (!k) continue;
        uint32_t *sub = (uint32_t *)malloc((size_t)k * k * sizeof(uint32_t));
        if (!sub) return -1;
        for (uint32_t a = 0; a < k; ++a)
            for (uint32_t b = 0; b < k; ++b) sub[a * k + b] = D[(size_t)members[a] * n + members[b]];
        uint64_t cl;
        uint32_t lr[64];
        const int rc = orc_route_held_karp(k, sub, &cl, lr);
        free(sub);
        if (rc) return -1;
        for (uint32_t t = 0; t < k; ++t) stops[at + t] = members[lr[t]];
        sizes[ncl++] = k;
        at += k;
    }
    if (orc_chain_routes(ncl, sizes, stops, n, D, 0, cost, route, NULL)) return -1;
    *m_used = mm;
    return 0;
}

int orc_order_routes_clustered(uint32_t num_orders, const uint32_t *pick_off, const uint32_t *D, const int32_t *xy,
                               uint32_t m, uint32_t max_cluster, uint32_t m_max, uint64_t *cost, uint32_t *route,
                               uint32_t *m_used, int nthreads)
{
    uint64_t *base = (uint64_t *)malloc(((size_t)num_orders + 1) * sizeof(uint64_t));
    if (!base) return -1;
    base[0] = 0;
    for (uint32_t o = 0; o < num_orders; ++o) {
        const uint64_t P = pick_off[o + 1] - pick_off[o];
        base[o + 1] = base[o] + P * P;
    }
    int bad = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
#endif
    for (int64_t o = 0; o < (int64_t)num_orders; ++o) {
        const uint32_t a = pick_off[o], P = pick_off[o + 1] - a;
        if (orc_route_clustered(P, D + base[o], xy + 2 * (size_t)a, m, max_cluster, m_max, cost + o, route + a,
                                m_used + o) != 0)
            bad |= 1;
    }
    free(base);
    return bad ? -1 : 0;
}
