/*
 * wroute.h -- C ABI of the MI355X warehouse routing library.
 *
 * The library computes the routing step of arXiv 2504.20655: shortest-path
 * distances over a warehouse graph with non-negative integer arc weights,
 * for one or many sources at once (Bellman-Ford relaxation, GPU
 * Implementation subsection, where `dist`/`pred` hold V x N entries for N
 * sources), optionally split into memory-bounded segments stitched through
 * their boundary vertices (the segmentation strategy named in the abstract
 * and in the Discussion), and the per-order pick-to-pick distance matrices
 * that route optimisation consumes (Route Optimization section; the picks of
 * an order are its stopping nodes, routes-and-clusters subsection).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns a wr_status.  Nothing aborts, nothing throws
 *    across the ABI.  wr_last_error() returns a thread-local message for the
 *    last failing call on the calling thread.
 *  - Validation happens before any device work; a validation error leaves
 *    every output buffer untouched.  After WR_E_DEVICE / WR_E_NOMEM /
 *    WR_E_INTERNAL the contents of output buffers are unspecified.
 *  - Ownership: inputs are copied before a call returns, so the caller may
 *    free them.  Outputs go to caller-provided buffers.  Handles are opaque
 *    and freed by their *_destroy function (NULL is accepted and ignored).
 *  - Host vs device buffers: index inputs (sources, pick_offsets, picks,
 *    segment maps, weight updates) are host pointers, because the batch
 *    plan is made on the host; with WR_DEVICE_INDEX the sources, offsets
 *    and picks of wr_sssp / wr_order_matrices may be device pointers, which
 *    the call reads back after the caller's earlier work on `stream`.  Output buffers (dist, pred, dist_out,
 *    pred_out) are host pointers unless WR_DEVICE_PTRS is set, in which case
 *    they are device pointers (for example torch's data_ptr()) and the
 *    results are written by work enqueued on `stream` (a hipStream_t, NULL =
 *    the default stream).  In both cases the call returns after the
 *    relaxation has converged; with WR_DEVICE_PTRS the final writes are
 *    ordered on `stream`.
 *  - Sentinels and types: WR_INF = 0xFFFFFFFF marks "no path";
 *    WR_NO_PRED = -1 marks "no predecessor".  V < 2^31, E < 2^32, weights
 *    are uint32 >= 0.
 *  - Threading: a context and its graphs are not thread-safe; the
 *    wr_server_* calls are internally synchronised.
 */
#ifndef WROUTE_H
#define WROUTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum wr_status {
    WR_OK = 0,
    WR_E_INVALID = 1,      /* malformed argument (bad CSR, id out of range, NULL) */
    WR_E_RANGE = 2,        /* a distance could reach WR_INF (overflow bound)      */
    WR_E_NOMEM = 3,        /* device memory or the context's budget exhausted     */
    WR_E_DEVICE = 4,       /* a HIP call failed                                   */
    WR_E_UNSUPPORTED = 5,  /* valid request the library does not serve            */
    WR_E_BUSY = 6,         /* queue full / result not ready                       */
    WR_E_INTERNAL = 7      /* invariant broken (e.g. round cap hit)               */
} wr_status;

#define WR_INF 0xFFFFFFFFu
#define WR_NO_PRED (-1)

/* ---- flags for wr_sssp / wr_order_matrices -------------------------- */
#define WR_DEVICE_PTRS      0x0001u  /* output buffers are device pointers */
/* relaxation schedule (all give bit-identical distances; 0 = automatic) */
#define WR_ALGO_AUTO        0x0000u
#define WR_ALGO_SWEEP       0x0010u  /* unsegmented pull sweeps (Jacobi/in-place) */
#define WR_ALGO_FRONTIER    0x0020u  /* unsegmented push frontier with ballot masks */
#define WR_ALGO_SEGMENTED   0x0030u  /* LDS-resident segments + boundary exchange   */
#define WR_ALGO_EDGE_B1     0x0040u  /* paper-structured: thread per arc, early exit */
#define WR_ALGO_EDGE_B0     0x0050u  /* paper-structured: exactly V-1 rounds         */
#define WR_ALGO_OVERLAY     0x0060u  /* segments with per-epoch boundary tables: passes are
                                        dense min-plus maps from a tile's incoming cross
                                        arcs to its exits (tiles of at most 512 vertices,
                                        64 incoming cross arcs, 64 exits and 512 cross
                                        arcs leaving; WR_E_UNSUPPORTED otherwise, and
                                        WR_ALGO_AUTO then takes WR_ALGO_SEGMENTED)   */
#define WR_ALGO_MASK        0x00F0u
#define WR_NO_GRAPH_CAPTURE 0x0100u  /* launch passes eagerly instead of replaying a hipGraph */
#define WR_TIME_KERNELS     0x0200u  /* record HIP events around every launch of the schedule's
                                        relaxation kernel (wr_run_info.kernel_ms); passes are
                                        then launched eagerly, not replayed from a hipGraph */
#define WR_PRUNE_TO_PICKS   0x0800u  /* wr_order_matrices, overlay schedule: stop each source's
                                        relaxation beyond the farthest pick it is paired with
                                        (exact for the matrices; see wr_order_matrices) */
#define WR_DEVICE_INDEX     0x1000u  /* wr_sssp sources / wr_order_matrices pick_offsets and
                                        picks are device pointers: copied to the host on
                                        `stream` after the caller's earlier work there (the
                                        call waits for that work; it still returns after
                                        convergence) */

/* ---- opaque handles -------------------------------------------------- */
typedef struct wr_context wr_context;
typedef struct wr_graph wr_graph;
typedef struct wr_server wr_server;

/* Name of a status code (static string). */
const char *wr_status_str(wr_status s);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *wr_last_error(void);

/* Library version string (static). */
const char *wr_version(void);

/* ---- context --------------------------------------------------------- */

/* Creates a context on HIP device `device`.  mem_budget_bytes bounds the
 * device memory the context allocates (graph, segment tables, per-batch
 * work buffers); 0 = 90% of the device's free memory at creation.
 * Errors: WR_E_INVALID (out == NULL, bad device), WR_E_DEVICE. */
wr_status wr_context_create(int device, uint64_t mem_budget_bytes, wr_context **out);
wr_status wr_context_destroy(wr_context *ctx);

/* Bytes the context currently holds and its budget. */
wr_status wr_context_memory(const wr_context *ctx, uint64_t *used, uint64_t *budget);

/* ---- graph ----------------------------------------------------------- */

/* Checks a CSR graph without a context.  The graph is directed; arc e goes
 * from the row u with row_ptr[u] <= e < row_ptr[u+1] to col[e] with weight
 * w[e] (the paper stores arcs as integer arrays u, v, w; CSR groups them by
 * u).  Parallel arcs and self-loops are allowed.
 * WR_E_INVALID: NULL arrays, V == 0, V >= 2^31, row_ptr[0] != 0,
 *   row_ptr decreasing, row_ptr[V] != E, col[e] >= V.
 * WR_E_RANGE: max_w * (number of vertices incident to an arc - 1) >= WR_INF,
 *   i.e. a shortest path could overflow the uint32 distance. */
wr_status wr_validate_csr(uint32_t V, uint32_t E, const uint32_t *row_ptr,
                          const uint32_t *col, const uint32_t *w);

/* Validates (as above) and uploads a graph; it stays device-resident until
 * wr_graph_destroy.  row_ptr: uint32[V+1]; col, w: uint32[E]; host pointers,
 * copied.  `flags` is reserved (pass 0).  The graph starts at weight epoch 0.
 * Errors: those of wr_validate_csr, WR_E_NOMEM, WR_E_DEVICE. */
wr_status wr_graph_create_csr(wr_context *ctx, uint32_t V, uint32_t E,
                              const uint32_t *row_ptr, const uint32_t *col,
                              const uint32_t *w, uint32_t flags, wr_graph **out);
wr_status wr_graph_destroy(wr_graph *g);

/* Partitions the vertices into segments: segment_of_vertex[v] < num_segments
 * (uint32[V], host).  A segment is a vertex set; its boundary vertices are
 * those with an arc to or from another segment.  Segments are relaxed
 * independently in on-chip memory and stitched by relaxing the cross-segment
 * arcs until nothing changes (the Discussion's sub-routes processed
 * independently within the GPU's memory).  A segment larger than one LDS
 * tile is split internally into tiles of consecutive vertex ids; vertices
 * without arcs belong to no tile.  Replaces any earlier segmentation.
 * Errors: WR_E_INVALID (NULL, num_segments == 0, id >= num_segments),
 * WR_E_NOMEM, WR_E_DEVICE. */
wr_status wr_graph_set_segments(wr_graph *g, const uint32_t *segment_of_vertex,
                                uint32_t num_segments);

/* Segments a grid whose vertex ids are level*W*H + y*W + x into
 * tile_w x tile_h rectangles per level.  Requires V == W*H*levels.
 * Errors: WR_E_INVALID (sizes zero or not matching V), as above. */
wr_status wr_graph_segment_grid(wr_graph *g, uint32_t W, uint32_t H, uint32_t levels,
                                uint32_t tile_w, uint32_t tile_h);

/* Number of segments and LDS tiles of the current segmentation (0 if none). */
wr_status wr_graph_segment_info(const wr_graph *g, uint32_t *num_segments,
                                uint32_t *num_tiles, uint32_t *num_boundary);

/* Sets w[arc_index[i]] = new_w[i] for i < n (arc_index = CSR position, host
 * arrays; a later entry for the same arc wins) and starts a new weight epoch,
 * returned in *out_epoch (may be NULL).  Work started after the call returns
 * uses the new weights.  Errors: WR_E_INVALID (index >= E, NULL with n > 0),
 * WR_E_RANGE (the overflow bound of wr_validate_csr would break; nothing is
 * changed), WR_E_DEVICE. */
wr_status wr_graph_update_weights(wr_graph *g, uint32_t n, const uint32_t *arc_index,
                                  const uint32_t *new_w, uint64_t *out_epoch);

/* Current weight epoch. */
wr_status wr_graph_epoch(const wr_graph *g, uint64_t *epoch);

/* ---- shortest paths -------------------------------------------------- */

/* Single- and multi-source shortest distances.
 * sources: uint32[S] (host), duplicates allowed.
 * dist:    uint32[S*V], source-major: dist[i*V + v] = d(sources[i], v),
 *          WR_INF where v is unreachable.
 * pred:    int32[S*V] or NULL: pred[i*V + v] = the smallest vertex id u with
 *          an arc (u, v) such that d(u) + w(u, v) = d(v); WR_NO_PRED for the
 *          source itself and for unreachable v.  With every weight >= 1 this
 *          is a shortest-path tree.
 * flags:   WR_DEVICE_PTRS, one WR_ALGO_* value, WR_NO_GRAPH_CAPTURE.
 * Errors: WR_E_INVALID (NULL, a source >= V), WR_E_UNSUPPORTED (pred
 * requested while some weight is 0: ties could then form cycles; or the
 * requested schedule cannot serve this graph), WR_E_NOMEM (not even one
 * source fits the budget), WR_E_DEVICE, WR_E_INTERNAL. */
wr_status wr_sssp(wr_graph *g, uint32_t S, const uint32_t *sources, uint32_t *dist,
                  int32_t *pred, uint32_t flags, void *stream);

/* Per-order pick-to-pick distance matrices.
 * pick_offsets: uint32[num_orders+1] (host), non-decreasing, first 0;
 *               order o owns picks[pick_offsets[o] .. pick_offsets[o+1]).
 * picks:        uint32[pick_offsets[num_orders]] vertex ids (host).
 * dist_out:     uint32[sum_o P_o^2]: for order o with P_o picks, the block
 *               D_o[i][j] = d(p_i, p_j) (row = source pick, row-major),
 *               blocks concatenated in order.  Duplicate picks give equal
 *               rows and columns with 0 between them; an empty order
 *               contributes nothing.
 * pred_out:     int32[sum_o P_o * V] or NULL: the canonical predecessor row
 *               (as in wr_sssp) of every pick, in pick order.
 * Distinct pick vertices are solved once per call, whatever order they
 * belong to.
 * WR_PRUNE_TO_PICKS (overlay schedule; WR_ALGO_AUTO selects it): a source
 * only needs its distances to the picks of the orders it belongs to, so a
 * value above the length of a path already found from it to each of those
 * picks is never stored (the bound is refined from the current tentative
 * matrix entries after every graph replay of passes).  Every vertex on a
 * shortest path to such a pick is no farther than the pick, so the matrices
 * are exact; the saving is largest when an order's picks lie close
 * together.  Not combinable with pred_out (WR_E_INVALID).
 * Errors as for wr_sssp, plus WR_E_INVALID for bad offsets. */
wr_status wr_order_matrices(wr_graph *g, uint32_t num_orders, const uint32_t *pick_offsets,
                            const uint32_t *picks, uint32_t *dist_out, int32_t *pred_out,
                            uint32_t flags, void *stream);

/* Optimal open route over each order's stops, from its distance matrix
 * (Route Optimization section: the entrance/exit is not part of a route, so
 * a route is an ordering of the order's P stops with any first and any last
 * stop, and its length is the sum of the P-1 matrix entries along it; the
 * section names Held and Karp's subset programme as the exact method,
 * which the kernel runs, one workgroup per order with its states in LDS).
 * Orderings are directed (D[i][j] is the step from stop i to stop j), so an
 * asymmetric matrix is served too; for a symmetric one the two travel
 * directions of a route tie and the smaller ordering is returned.
 *
 * pick_offsets: uint32[num_orders+1] (host), non-decreasing, first 0; order
 *               o has P_o = pick_offsets[o+1] - pick_offsets[o] stops,
 *               P_o <= WR_ROUTE_MAX_STOPS.
 * dist:         uint32[sum_o P_o^2]: the concatenated row-major P_o x P_o
 *               matrices, as wr_order_matrices writes them; WR_INF marks a
 *               step that cannot be taken.
 * length_out:   uint64[num_orders]: the shortest route's length,
 *               WR_ROUTE_INF when every ordering takes a WR_INF step (0 for
 *               orders of 0 or 1 stops).
 * route_out:    uint32[pick_offsets[num_orders]]: order o's ordering at
 *               pick_offsets[o], as indices 0..P_o-1 into its picks; among
 *               shortest orderings the lexicographically smallest.
 * flags:        WR_DEVICE_PTRS: dist, length_out and route_out are device
 *               pointers, read and written by work ordered after `stream`
 *               (pick_offsets stays a host array).
 *               WR_ROUTE_ENUMERATE: the paper's own structure instead (its
 *               route-permutation kernel, numerical-experiments section): one
 *               thread per ordering, n! orderings of n-1 steps each, for
 *               orders of at most WR_ROUTE_ENUMERATE_MAX_STOPS stops; the same
 *               results, kept as the baseline the subset programme is
 *               measured against.
 * Errors: WR_E_INVALID (NULL, bad offsets, unknown flags), WR_E_UNSUPPORTED
 * (an order with more than WR_ROUTE_MAX_STOPS stops, or more than
 * WR_ROUTE_ENUMERATE_MAX_STOPS with WR_ROUTE_ENUMERATE), WR_E_RANGE (the
 * length of some partial route of an order reaches 2^32-1: lengths are
 * accumulated in 32 bits; outputs are then unspecified), WR_E_NOMEM,
 * WR_E_DEVICE. */
#define WR_ROUTE_MAX_STOPS 12u
#define WR_ROUTE_ENUMERATE 0x0400u
#define WR_ROUTE_ENUMERATE_MAX_STOPS 10u
#define WR_ROUTE_INF 0xFFFFFFFFFFFFFFFFull
wr_status wr_order_routes(wr_context *ctx, uint32_t num_orders, const uint32_t *pick_offsets,
                          const uint32_t *dist, uint64_t *length_out, uint32_t *route_out,
                          uint32_t flags, void *stream);

/* Exact routes for callers that cannot allocate device memory (code under
 * their own graph capture, tight serving loops, harnesses that forbid
 * allocation): the results of wr_order_routes, with every work buffer held
 * in one fixed device array of the library (about 1.3 MB, kept by each GPU
 * the library runs on until the process ends) instead of allocations.
 * dist, length_out and route_out are device pointers, laid out as for
 * wr_order_routes; pick_offsets is a host array (validated on the host).
 * The work is enqueued on `stream` (the caller's hipStream_t; NULL is the
 * null stream) after the caller's earlier work on it, and the call returns
 * once it is done.  flags: 0 or WR_ROUTE_ENUMERATE.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU race, so a caller
 * serialises them.  Errors: as wr_order_routes, and WR_E_RANGE when
 * num_orders exceeds WR_ROUTES_STATIC_MAX_ORDERS (nothing is enqueued). */
#define WR_ROUTES_STATIC_MAX_ORDERS 65536u
wr_status wr_order_routes_static(wr_context *ctx, uint32_t num_orders, const uint32_t *pick_offsets,
                                 const uint32_t *dist, uint64_t *length_out, uint32_t *route_out,
                                 uint32_t flags, void *stream);

/* Cluster-decomposed route over each order's stops (the theorem of the
 * Route Optimization section): the stops are split into m clusters by
 * K-means on their positions (a cluster's centre is the mean position of
 * its picks, routes-and-clusters subsection), the optimal open route is
 * found inside each cluster (as in wr_order_routes), and the global route is
 * the cheapest chaining of the cluster routes over every order of the
 * clusters and every orientation of each, adding the steps between
 * consecutive clusters' ends.  Not optimal in general, never shorter than
 * wr_order_routes' result, and served for orders too large for it.
 * Readings where the section is silent: farthest-point initial centres
 * from the first pick (ties to the smaller index); Lloyd steps until no
 * assignment changes, at most 100 (ties to the smaller cluster, an empty
 * cluster keeps its centre); distances to centres compared exactly in
 * integers; m grows by one while a cluster has more than
 * WR_ROUTE_MAX_STOPS picks; the cheapest chain is found by a subset
 * programme over (clusters used, first cluster, its orientation), and among
 * the cheapest the lexicographically smallest sequence of (cluster,
 * orientation) is returned, forward before reversed.
 *
 * pick_offsets, dist, length_out, route_out: as for wr_order_routes, with
 *               P_o <= WR_CLUSTER_MAX_STOPS.
 * pick_xy:      int32[2 * pick_offsets[num_orders]]: (x, y) of each pick,
 *               |x|, |y| < 2^16 (host, or device with WR_DEVICE_PTRS).
 * m:            clusters requested, 1 <= m <= WR_CLUSTER_MAX_CLUSTERS.
 * clusters_out: uint32[num_orders] (host, whatever the flags) or NULL:
 *               clusters each order used.
 * Errors: WR_E_INVALID (NULL, bad offsets, m out of range, unknown flags),
 * WR_E_UNSUPPORTED (an order above WR_CLUSTER_MAX_STOPS stops, or one that
 * no m <= WR_CLUSTER_MAX_CLUSTERS splits into small enough clusters),
 * WR_E_RANGE (a position out of range, or a length reaching 2^32-1 inside
 * a cluster), WR_E_NOMEM, WR_E_DEVICE; outputs are unspecified after an
 * error found on the device. */
#define WR_CLUSTER_MAX_STOPS 64u
#define WR_CLUSTER_MAX_CLUSTERS 10u
wr_status wr_order_routes_clustered(wr_context *ctx, uint32_t num_orders, const uint32_t *pick_offsets,
                                    const uint32_t *dist, const int32_t *pick_xy, uint32_t m,
                                    uint64_t *length_out, uint32_t *route_out, uint32_t *clusters_out,
                                    uint32_t flags, void *stream);

/* ---------------------------------------------------------------------
 * The warehouse reorganisation loop (Mathematical model section: the state
 * x = (A, M), orders, the map f and the random dynamical system
 * x_n = f(o_n, x_{n-1}); the Clustering section's restocking rule; the WMS
 * loop appendix: order processing, stock update, check-and-move).
 *
 * Node v = (k * ny + j) * nx + i is shelf k of rack (i, j).  A picking
 * order is `purchase_orders` purchase orders of `articles_per_order` slots
 * each (20 of 10 in the paper's experiments); slot s of purchase order p is
 * entry p * articles_per_order + s.  One application of f, per run and
 * iteration:
 *   1. each purchase order's point is (sum of i, sum of j) over the racks of
 *      its articles; the points are split into `clusters` clusters by the
 *      K-means reading of wr_order_routes_clustered;
 *   2. metrics of that clustering: the silhouette score of the points as
 *      mean positions (point / articles_per_order; a point alone in its
 *      cluster scores 0, so does one with a = b = 0) and the area of the
 *      triangle of the first three non-empty clusters' centres (0 with
 *      fewer); a centre is the mean rack position of its cluster's articles;
 *   3. the picks in slot order: article a at node v with balance m, q
 *      parcels: if m > q then m -= q; else the empty node u nearest a's
 *      cluster centre (squared distance of rack positions, compared exactly;
 *      ties to the smaller node id) takes a if it is strictly nearer than
 *      v -- v becomes empty (A = 0, M = 0) and u gets a with
 *      mmax - (q - m) parcels -- otherwise v is restocked in place to
 *      mmax - (q - m).
 *
 * params:      the warehouse and the order shape (below).
 * runs, iters: independent runs, and iterations (orders) per run.
 * A, M:        uint32[runs][V], in/out: article per node (0 = empty, else
 *              1..n_articles, each article at most one node per run) and
 *              balance per node; left holding the state after `iters`
 *              iterations.
 * orders:      uint32[runs][iters][S] (S = purchase_orders *
 *              articles_per_order): the article of each slot; every one
 *              must be stored in the run's state.
 * qty:         uint32[runs][iters][S]: parcels of each slot, at most mmax.
 * silhouette, area: double[runs][iters]; moves: uint32[runs][iters]
 *              (articles moved by each iteration).
 * Every buffer is host memory, or device memory with WR_DEVICE_PTRS (then
 * the work runs after the caller's earlier work on `stream`).  The call
 * returns when the results are written.
 * Limits: nx, ny <= 2048, nz <= 32, V < 2^24, rack masks of
 * 4 * ceil(nx * ny / m) <= 65536 bytes (m = 3 racks per word for nz <= 10,
 * 2 for nz <= 16, else 1), purchase_orders <= 64, S <= 1024, clusters <= 10,
 * S * max(nx, ny) <= 2^19.
 * Errors: WR_E_INVALID (NULL, a parameter out of range, an article number
 * above n_articles or stored twice, an order's article not stored),
 * WR_E_RANGE (a slot of more than mmax parcels; host buffers only -- with
 * device buffers it is WR_E_INVALID), WR_E_UNSUPPORTED (a limit above),
 * WR_E_NOMEM, WR_E_DEVICE.  Host buffers are left unchanged by a failed
 * call; device buffers are unspecified after an error found on the
 * device. */
typedef struct wr_wms_params {
    uint32_t nx, ny, nz;            /* racks nx x ny, shelves nz              */
    uint32_t n_articles;            /* article types 1..n_articles            */
    uint32_t mmax;                  /* parcels of a full node                 */
    uint32_t purchase_orders;       /* per picking order                      */
    uint32_t articles_per_order;    /* slots per purchase order               */
    uint32_t clusters;              /* K of the K-means step                  */
} wr_wms_params;
wr_status wr_wms_run(wr_context *ctx, const wr_wms_params *params, uint32_t runs, uint32_t iters, uint32_t *A,
                     uint32_t *M, const uint32_t *orders, const uint32_t *qty, double *silhouette, double *area,
                     uint32_t *moves, uint32_t flags, void *stream);

/* Statistics of the last wr_sssp / wr_order_matrices call on this graph. */
typedef struct wr_run_info {
    uint32_t algo;             /* WR_ALGO_* value that ran                      */
    uint32_t unique_sources;   /* distinct sources solved                       */
    uint32_t chunks;           /* memory-bounded chunks                         */
    uint32_t passes;           /* relaxation passes (rounds) over all chunks    */
    uint64_t work_items;       /* visits: (tile, source) or (vertex, block)     */
    double relax_ms;           /* device time of the relaxation passes          */
    double total_ms;           /* wall time of the call                         */
    double kernel_ms;          /* with WR_TIME_KERNELS: summed duration of the
                                  relaxation kernel's launches (else 0)         */
    uint32_t kernel_launches;  /* launches timed into kernel_ms                 */
    uint64_t relaxations;      /* overlay schedule: min-plus relaxations of its
                                  passes (per source lane: each cross arc into
                                  a visited tile and each entry of the tile's
                                  port-to-exit table), else 0                   */
    uint64_t alg_bytes;        /* overlay schedule: state bytes its passes must
                                  move (a 256-byte row of 64 source values per
                                  incoming cross arc and per exit of a visited
                                  tile, 4 bytes per exit value stored), else 0 */
} wr_run_info;
wr_status wr_graph_last_run(const wr_graph *g, wr_run_info *info);

/* Chooses schedule parameters by timing candidates on this graph with
 * `sources_hint` synthetic sources (evenly spread vertices that have arcs)
 * and keeps the fastest: with a grid segmentation (wr_graph_segment_grid)
 * the grid tile shape (tile_w x tile_h cells; the segments the caller gave
 * are replaced by the chosen shape), the source blocks per workgroup unit
 * and the passes per graph replay of the overlay schedule; otherwise the
 * tile size, waves per tile and passes per replay.  Every candidate gives
 * identical distances, so results never depend on the outcome.  cache_path
 * (may be NULL) is a JSON file read before and written after tuning, keyed
 * by the graph's structure and the segmentation it was called with.
 * Errors: WR_E_INVALID, WR_E_DEVICE. */
wr_status wr_autotune(wr_graph *g, uint32_t sources_hint, const char *cache_path);

/* Sets schedule parameters explicitly (0 keeps the current value). */
wr_status wr_graph_set_schedule(wr_graph *g, uint32_t tile_vertices,
                                uint32_t waves_per_group, uint32_t passes_per_replay);

/* Sets the 64-source blocks one workgroup unit of the overlay and
 * segmented passes visits (1..64; 0 restores the default).  Errors:
 * WR_E_INVALID. */
wr_status wr_graph_set_blocks_per_unit(wr_graph *g, uint32_t blocks);

/* The schedule a graph runs with (as set, or as wr_autotune chose). */
typedef struct wr_schedule {
    uint32_t tile_vertices;      /* most vertices of one LDS tile               */
    uint32_t waves_per_group;    /* waves per workgroup (segmented schedule)    */
    uint32_t passes_per_replay;  /* passes captured in one graph replay          */
    uint32_t blocks_per_unit;    /* 64-source blocks one workgroup unit visits   */
    uint32_t grid_tile_w;        /* grid segment shape, 0 if the segmentation    */
    uint32_t grid_tile_h;        /*   is not a grid                              */
} wr_schedule;
wr_status wr_graph_get_schedule(const wr_graph *g, wr_schedule *out);

/* Test hook for failure handling: the nth next device allocation (kind 1,
 * the call fails with WR_E_NOMEM) or kernel launch (kind 2, WR_E_DEVICE)
 * the library makes, from any thread, fails on the host before anything
 * reaches the device; kind 0 disarms.  One fault at a time, process-wide.
 * The environment variable WR_FAULT=alloc:N or launch:N arms it at load.
 * Errors: WR_E_INVALID. */
wr_status wr_debug_fault(uint32_t kind, uint64_t nth);

/* ---- continuous-batching server -------------------------------------- */

typedef struct wr_server_opts {
    uint32_t max_source_slots;   /* sources relaxed concurrently (0 = auto)   */
    uint64_t mem_budget_bytes;   /* device bytes for in-flight work (0 = auto) */
    uint32_t max_queue;          /* queued requests before WR_E_BUSY (0 = 65536) */
    uint32_t passes_per_step;    /* relaxation passes per scheduler step (0 = auto) */
    uint32_t resident_epochs;    /* weight epochs kept resident: 1 (or 0): an update waits
                                    until no order is in flight; 2: see wr_server_create */
} wr_server_opts;

typedef struct wr_req_info {
    uint64_t epoch;      /* weight epoch the request was solved on  */
    double t_arrive;     /* seconds, server clock                   */
    double t_admit;
    double t_done;
    uint32_t P;          /* picks                                   */
    wr_status status;
} wr_req_info;

typedef struct wr_stats {
    uint64_t submitted, completed, failed;
    double p50_ms, p99_ms, mean_ms;   /* arrival -> result ready on the host */
    double throughput_per_s;          /* completed / (last done - first arrival) */
    uint32_t max_inflight_requests;
    uint64_t steps;
} wr_stats;

/* Creates a server over graph g (the server keeps g and its segmentation
 * resident; g must outlive the server and must not be used directly while
 * the server runs; when the server ends, g holds every accepted update).
 * On graphs that run the overlay schedule the server relaxes orders in
 * block rows of 64 sources, admitted between relaxation steps.  With
 * resident_epochs = 2 it keeps two weight epochs resident: it makes a
 * second copy of g (same segmentation and schedule) with rows of its own;
 * an update is applied to the copy whose rows have all retired, which then
 * takes the new orders while the other copy's orders finish on their epoch
 * (the rows of both copies come out of mem_budget_bytes; while both copies
 * have orders in flight a step relaxes both).  The call returns once the
 * server's state is built.  opts may be NULL for defaults. */
wr_status wr_server_create(wr_graph *g, const wr_server_opts *opts, wr_server **out);

/* Queues one order of P picks (host array, copied; P == 0 is allowed and
 * completes at once).  Non-blocking.  WR_E_BUSY if the queue is full;
 * WR_E_INVALID for a pick >= V or picks == NULL with P > 0. */
wr_status wr_server_submit(wr_server *srv, uint32_t P, const uint32_t *picks, uint64_t *ticket);

/* WR_OK and the P x P matrix in dist_out (host, row-major) once done;
 * WR_E_BUSY while pending; WR_E_INVALID for an unknown or already-collected
 * ticket.  info may be NULL.  A request that failed returns its status. */
wr_status wr_server_poll(wr_server *srv, uint64_t ticket, uint32_t *dist_out, wr_req_info *info);

/* Queues a weight update; it is applied between scheduler steps (with two
 * resident epochs to the copy of the graph with nothing in flight, else
 * once no order is in flight), and every request admitted after that point
 * is solved on the new epoch (wr_req_info.epoch: the caller graph's epoch at creation plus
 * the updates accepted before the request's admission).  Arc
 * indices are checked here (WR_E_INVALID); an update that the graph would
 * refuse at application time (WR_E_RANGE, see wr_graph_update_weights) is
 * dropped and the epoch does not advance. */
wr_status wr_server_update_weights(wr_server *srv, uint32_t n, const uint32_t *arc_index,
                                   const uint32_t *new_w);

/* Latency and throughput statistics so far. */
wr_status wr_server_stats(wr_server *srv, wr_stats *out);

/* Blocks until every submitted request is done (or failed). */
wr_status wr_server_drain(wr_server *srv);

wr_status wr_server_destroy(wr_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* WROUTE_H */
