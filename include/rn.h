/*
 * rn.h -- C ABI of the network-distance join library (librn).
 *
 * The library answers the two proximity queries of "Parallelized
 * Proximity-Based Query Processing Methods for Road Networks" (arXiv 1607.07696)
 * on one AMD Instinct GPU (gfx950):
 *
 *   theta-join (Abstract; Section 1; Section 4, opening paragraph): given two
 *     disjoint node sets R and S of a road network and a distance bound theta,
 *     every pair (u, v) with u in R, v in S and network distance
 *     dist(u,v) <= theta.  dist is the length of a shortest directed path from
 *     u to v over the graph's arcs (R precedes S: distances are taken from u to
 *     v; on an undirected graph stored as two arcs per edge this is moot).
 *
 *   k closest pairs (Abstract; Section 1; Section 6): the k pairs (u, v),
 *     u in R, v in S, with no pair left out closer than a pair kept.  Section 4
 *     frames both queries as one interface (k results within theta); an
 *     unbounded k gives the theta-join.
 *
 * Results are exact: integer weights, uint32 distances, and every result list
 * sorted by (dist, u, v) ascending on the caller's vertex ids.  That order also
 * breaks ties among equal distances, which the paper leaves open, so the
 * k-closest-pairs answer is unique.  A path of length >= 2^32 - 1 counts as
 * unreachable; unreachable pairs are never reported.
 *
 * Memory spaces.  Graph arrays handed to rn_graph_load and rn_partition_host
 * are HOST pointers.  The R, S and out arrays of the join calls are DEVICE
 * pointers (for example torch tensors' data_ptr() on the current device);
 * counts returned through int64_t* are HOST pointers.  The library copies what
 * it needs and never takes ownership of caller memory.
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * All device work of a call is enqueued on it; the join calls return only after
 * that work has finished (they must report the result count).
 *
 * Threads.  Calls on different rn_graph handles may run concurrently from
 * different host threads.  Calls on one handle must not overlap: each handle
 * owns one set of query buffers (RN_ERR_BUSY is returned if they would).
 *
 * Errors.  Every call returns an rn_status.  No C++ exception crosses this ABI.
 * rn_last_error() returns a message describing the calling thread's most
 * recent failure.
 */
#ifndef RN_H
#define RN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rn_status;
#define RN_OK            0
#define RN_ERR_ARG      (-1)   /* invalid argument (bad id, duplicate, R and S overlap, ...) */
#define RN_ERR_NOMEM    (-2)   /* host or device allocation failed */
#define RN_ERR_CAPACITY (-3)   /* output buffer too small; *n_out holds the required count */
#define RN_ERR_DEVICE   (-4)   /* HIP runtime error (no device, launch failure, ...) */
#define RN_ERR_BUSY     (-5)   /* another call is using this handle */

/* One result pair: u in R, v in S, dist = dist(u, v).  12 bytes, no padding. */
typedef struct rn_pair {
    int32_t u;
    int32_t v;
    uint32_t dist;
} rn_pair;

/* Opaque handle: a graph resident in device memory plus its query buffers. */
typedef struct rn_graph rn_graph;

/*
 * rn_graph_load -- copy a CSR graph to the current HIP device and keep it there.
 *
 * The road network of Section 1 as a directed graph in CSR form: the out-arcs of
 * vertex x are arcs row_ptr[x] .. row_ptr[x+1]-1; arc a leads to col[a] with
 * weight w[a].  An undirected road stores each edge as two arcs of equal weight.
 *   V        number of vertices, 1 <= V < 2^31 - 1
 *   A        number of arcs, 0 <= A < 2^31
 *   row_ptr  host int32[V+1]: row_ptr[0] = 0, non-decreasing, row_ptr[V] = A
 *   col      host int32[A]:   0 <= col[a] < V
 *   w        host uint32[A]:  any value (zero weights, self-loops and parallel
 *            arcs are accepted)
 *   out      receives the handle; *out is NULL on failure
 * The caller keeps ownership of its arrays.  Errors: RN_ERR_ARG on a malformed
 * CSR or null pointer, RN_ERR_NOMEM, RN_ERR_DEVICE.
 * Node coordinates are not taken: both queries are defined on network
 * distance alone (Section 1), so nothing on the device would read them.
 */
rn_status rn_graph_load(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col,
                        const uint32_t *w, rn_graph **out);

/*
 * rn_objects_graph -- objects on the edges of a road network (Section 1:
 * objects that move along edges, given by their distances from the two ends
 * of their edge, may take the place of nodes in R or S).  Returns a new
 * handle whose graph is graph `graph` of g with object i inserted into its
 * edge as vertex V + i (V: that graph's vertex count); every join call then
 * takes objects, nodes or both in R and S, and the pairs name object i as
 * V + i.  Snapshot semantics: a moved object needs a new handle.
 *   arc, offset  host int32[n], uint32[n]: object i lies on arc arc[i] =
 *            (a -> b, weight w) of that graph (local arc index, 0 .. A-1), at
 *            distance offset[i] <= w from a
 * The object's edge is the road of that arc; parallel arcs of equal ends and
 * weight are one road (the first of them carries the object), and the road
 * is two-way when an arc b -> a of weight w exists (the first such arc, not
 * the road's own arc for a loop, is the same road traversed back, so an
 * object named on it lies on the same road at w - offset from a).  The road's arcs become a chain through its
 * objects in order of position: one-way, objects move and are reached in the
 * arc's direction only; two-way, both ways.  Distances between the graph's
 * own vertices do not change.  The caller keeps its arrays; free the new
 * handle with rn_graph_free.  Errors: RN_ERR_ARG (bad handle, index, arc or
 * offset), RN_ERR_NOMEM, RN_ERR_DEVICE.
 */
rn_status rn_objects_graph(const rn_graph *g, int32_t graph, const int32_t *arc, const uint32_t *offset, int32_t n,
                           rn_graph **out);

/* Free a handle and all its device memory.  NULL is accepted. */
void rn_graph_free(rn_graph *g);

/* Number of vertices / arcs of a loaded graph, summed over its graphs (0 for NULL). */
int32_t rn_graph_num_vertices(const rn_graph *g);
int64_t rn_graph_num_arcs(const rn_graph *g);

/*
 * rn_partition_host -- the paper's heuristic recursive bisection (Section 3,
 * Algorithm 1 with the smoothing of Equations (1)-(2)) on a host CSR.
 *
 * Each bisection grows two clusters from two seed vertices, always expanding
 * the cluster whose lightest frontier edge (after smoothing by alpha) is the
 * lighter; the recursion stops at parts of at most max_leaf vertices.  Seeds
 * are a double-sweep pseudo-diameter of the part (the paper leaves them open).
 * Arc directions are ignored (each arc is treated as an undirected edge).
 *   alpha     smoothing in [0, 1]; 0 = plain edge weights
 *   max_leaf  largest leaf part, >= 1
 *   part_out  host int32[V] or NULL: leaf id of each vertex; leaf ids follow a
 *             left-to-right walk of the recursion
 *   order_out host int32[V] or NULL: the vertices listed leaf by leaf
 * Errors: RN_ERR_ARG (bad CSR, alpha outside [0,1], max_leaf < 1), RN_ERR_NOMEM.
 */
rn_status rn_partition_host(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col,
                            const uint32_t *w, float alpha, int32_t max_leaf,
                            int32_t *part_out, int32_t *order_out);

/*
 * rn_partition -- partition each graph of a handle (as rn_partition_host) and
 * renumber the handle's device copy of a graph in the leaf-by-leaf vertex
 * order where that keeps the two ends of its arcs closer together (mean id
 * distance over the arcs) than the numbering it was loaded with: the arcs of
 * the vertices of one leaf then sit next to each other in memory, and joins
 * visit their sources leaf by leaf (well-separated regions, Section 3).  A
 * graph loaded with a numbering that is already local keeps it.  Ids at the
 * boundary stay the caller's: R, S and the pairs of every call use the
 * numbering the graph was loaded with.  Join results never depend on it.
 * Waits for the device; do not call it while work of the handle (a plan
 * replay) is running (a server holds the handle: RN_ERR_BUSY).
 *   part_out  host int32[total V] or NULL: the leaf id of each vertex, graph
 *             after graph; leaf ids are numbered on across the graphs
 */
rn_status rn_partition(rn_graph *g, float alpha, int32_t max_leaf, int32_t *part_out);

/* 1 if rn_partition renumbered the device copy of graph `graph` of the handle
 * in leaf order, else 0 (also for a bad handle or index). */
int32_t rn_graph_renumbered(const rn_graph *g, int32_t graph);

/*
 * rn_dist_join -- the theta-join (on graph 0 of the handle); the query as the
 * Abstract and the opening of Section 4 define it: pairs of R x S whose
 * network distance is within theta.
 *   R, nR   device int32[nR], nR >= 1: the left set; ids in [0, V), no duplicates
 *   S, nS   device int32[nS], nS >= 1: the right set; ids in [0, V), no
 *           duplicates, disjoint from R (the paper's sets are disjoint)
 *   theta   distance bound, inclusive, 0 <= theta <= 2^32 - 2
 *   out     device rn_pair[cap] (may be NULL when cap == 0)
 *   n_out   host: number of pairs found
 * On RN_OK, out[0 .. *n_out) holds every (u, v, dist(u,v)) with dist <= theta,
 * sorted by (dist, u, v).  If *n_out would exceed cap, RN_ERR_CAPACITY is
 * returned with *n_out set to the required count and out left unspecified
 * (call again with a larger buffer).  RN_ERR_ARG on a bad id, a duplicate, an
 * overlap of R and S, or theta out of range.
 */
rn_status rn_dist_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                       uint32_t theta, rn_pair *out, int64_t cap, int64_t *n_out, void *stream);

/*
 * rn_kcp_join -- the k-closest-pairs join (on graph 0 of the handle); the
 * query as the Abstract and Section 1 define it: k pairs of R x S such that no
 * pair left out is closer than a pair returned.
 *   R, nR, S, nS  as for rn_dist_join
 *   k       1 <= k <= 2^24
 *   out     device rn_pair[cap]; cap >= min(k, nR * nS) always suffices
 *   n_out   host: number of pairs returned = min(k, number of reachable pairs)
 * On RN_OK, out[0 .. *n_out) holds the first pairs of the (dist, u, v) order
 * over all reachable (u, v), u in R, v in S.  RN_ERR_CAPACITY (with the count)
 * if cap is too small; RN_ERR_ARG as for rn_dist_join or k out of range.
 */
rn_status rn_kcp_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                      int32_t k, rn_pair *out, int64_t cap, int64_t *n_out, void *stream);

/*
 * Tuning knobs of a handle (they never change results).
 *   delta        bucket width of the bucketed relaxation; 0 = one bucket
 *                (a FIFO of pending vertices).  Default chosen at load.  Used by
 *                tables up to 2^11 entries; larger tables, searched by several
 *                waves together, always use one bucket.
 *   hash_log2    log2 of the per-source LDS table size tried first (8..14);
 *                sources whose search outgrows it are re-run with larger ones.
 *                Until it is set, theta-joins start at 2^11 or at the size the
 *                expected ball for their theta needs, whichever is larger.
 * Pass a negative value to keep a knob's current setting.
 */
rn_status rn_set_tuning(rn_graph *g, int64_t delta, int32_t hash_log2);
rn_status rn_get_tuning(const rn_graph *g, uint32_t *delta, int32_t *hash_log2);

/*
 * ---- Several graphs, many queries per call (the batched form).
 *
 * A handle may hold several independent graphs.  rn_join_batch runs any mix
 * of theta-joins and k-closest-pairs queries over them as one launch sequence
 * on one stream: the searches of all queries share the device at once, so
 * many small queries cost about as much as one large one.
 */

/*
 * rn_graph_load_many -- load n graphs into one handle (graph i keeps its own
 * vertex ids 0 .. V[i]-1).  Each graph is a CSR as for rn_graph_load; the
 * arrays are host pointers.  The total vertex count must stay below 2^31 - 1
 * and the total arc count below 2^31.  rn_graph_load is this call with n = 1.
 */
rn_status rn_graph_load_many(int32_t n, const int32_t *V, const int64_t *A, const int32_t *const *row_ptr,
                             const int32_t *const *col, const uint32_t *const *w, rn_graph **out);

/* Number of graphs in a handle (0 for NULL), and the size of graph i. */
int32_t rn_graph_count(const rn_graph *g);
rn_status rn_graph_size(const rn_graph *g, int32_t i, int32_t *V, int64_t *A);

#define RN_DELTA_DEFAULT 0xFFFFFFFFu   /* rn_query.delta: use the handle's setting */

/*
 * One query of a batch.
 *   R, S      device int32[nR], int32[nS]: node sets of graph `graph`, with the
 *             rules of rn_dist_join (ids in [0, V), no duplicates, disjoint)
 *   graph     index of the graph in the handle
 *   k         0: the theta-join (every pair within theta).  1 <= k <= 2^24:
 *             the first min(k, n) pairs of the (dist, u, v) order among the n
 *             pairs within theta, i.e. the k closest pairs within the bound
 *             (theta = 2^32 - 2 for the unbounded query; Section 4 casts both
 *             queries as "k results within theta")
 *   theta     distance bound, inclusive, <= 2^32 - 2
 *   delta     bucket width for this query's searches, or RN_DELTA_DEFAULT
 *   hash_log2 first on-chip table size for its searches (8..14),
 *             RN_TABLE_GLOBAL to run them in the global-memory tier from the
 *             start, or 0 for the default: the handle's setting for a
 *             theta-join, 8 for k > 0, and the global tier where the searches
 *             are sure to outgrow every on-chip table (a theta-join whose
 *             expected ball, about 2 (theta / mean arc weight)^2 vertices, is
 *             more than twice the largest table's capacity; a k-closest-pairs
 *             query that asks for at least half of its |R| |S| pairs on a
 *             graph of 2^16 vertices or more)
 * delta and hash_log2 never change results.
 */
#define RN_TABLE_GLOBAL 15
typedef struct rn_query {
    const int32_t *R;
    const int32_t *S;
    int32_t nR, nS;
    int32_t graph;
    int32_t k;
    uint32_t theta;
    uint32_t delta;
    int32_t hash_log2;
    int32_t flags;      /* 0, or RN_QUERY_FORWARD */
} rn_query;

/* rn_query.flags: run the searches from R even when S is smaller.  By default
 * a query whose S holds fewer vertices than its R searches from S over the
 * reversed arcs (dist(u, v) is the same path read backwards); the result is
 * identical either way.  Work counts (RN_PROFILE_WORK) follow the side searched. */
#define RN_QUERY_FORWARD 1

/*
 * rn_join_batch -- run nq queries (1 <= nq <= 65536) as one call.
 *   out       device rn_pair[cap]: query i's pairs are out[offsets[i] ..
 *             offsets[i+1]), sorted by (dist, u, v), ids local to its graph
 *   offsets   host int64[nq + 1]: segment starts; offsets[nq] = total pairs
 *   status    host int32[nq] or NULL: RN_OK, or RN_ERR_ARG for a query whose
 *             R or S is invalid (bad id, duplicate, overlap); such a query
 *             gets an empty segment and the others are still answered
 * Returns RN_OK when every query succeeded.  RN_ERR_CAPACITY when the total
 * exceeds cap: offsets then give the layout needed and out is left untouched.
 * RN_ERR_ARG when a query is malformed on the host side (bad graph index,
 * count, pointer, k or theta; nothing runs, status marks it) or invalid on
 * the device (status marks it; the valid queries' results are written).
 */
rn_status rn_join_batch(rn_graph *g, const rn_query *q, int32_t nq, rn_pair *out, int64_t cap, int64_t *offsets,
                        int32_t *status, void *stream);

/*
 * rn_autotune -- choose delta and hash_log2 for each query by timing a few
 * candidate settings on a sample of its sources (the first min(nR, sample)
 * entries of R) and keeping the one with the least relaxation time: delta in
 * {0, w_min, 4 w_min} times first table sizes (2^9..2^12 for theta-joins,
 * 2^8..2^10 for k > 0), plus the global tier from the start (RN_TABLE_GLOBAL)
 * with the default delta.  Writes q[i].delta and q[i].hash_log2; results
 * never depend on them.  The device work runs on `stream`.
 */
rn_status rn_autotune(rn_graph *g, rn_query *q, int32_t nq, int32_t sample, void *stream);

/*
 * Captured plans: a batch recorded once into a HIP graph and replayed with
 * one graph launch per run.  The plan keeps q[] (and so the device pointers
 * R, S) and out, cap as given; callers may change the contents of R, S
 * between runs but not their sizes.  A plan owns its own call buffers; runs
 * and other calls on the same handle must not overlap (RN_ERR_BUSY).
 *   rn_plan_create  runs the batch once on `stream` to size its buffers, then
 *                   captures it
 *   rn_plan_run     replays it on `stream` and reports as rn_join_batch (if a
 *                   run outgrows the record buffer it is re-sized, re-run and
 *                   re-captured)
 */
typedef struct rn_plan rn_plan;
rn_status rn_plan_create(rn_graph *g, const rn_query *q, int32_t nq, rn_pair *out, int64_t cap, void *stream,
                         rn_plan **plan);
rn_status rn_plan_run(rn_plan *p, int64_t *offsets, int32_t *status, void *stream);
void rn_plan_free(rn_plan *p);

/*
 * ---- Serving: a request server with continuous batching.
 *
 * A server keeps one graph of a handle resident and answers join requests
 * as they arrive.  A host thread of the library admits waiting requests, in
 * arrival order (with heavy_lane: in arrival order within the heavy and the
 * light requests, heavy ones one at a time, on the last lane first), into free lanes
 * whenever the estimated device footprint of
 * the requests in flight stays within hbm_budget (one request is admitted
 * whenever nothing is in flight, however large), and runs each lane's
 * requests as one batch (the launch sequence of rn_join_batch) on the lane's
 * own stream and buffers.  Requests that arrive while others are on the
 * device are admitted as lanes and budget free up, and their work overlaps
 * with the batches already running.  The budget covers what requests add
 * while in flight (their ids, records and output, estimated); the buffers
 * each lane keeps between batches, among them its global-tier search slots
 * (global_slots slots of 24 bytes per vertex each, allocated when the
 * server starts), are outside it and are reported in
 * rn_server_stats.device_bytes.  Each request's result is exactly the
 * result of the same query run alone.  The server holds the handle for its
 * lifetime: other calls on it return RN_ERR_BUSY until rn_server_free.
 */
typedef struct rn_server rn_server;

typedef struct rn_server_config {
    int32_t graph;          /* graph of the handle the requests address */
    int32_t lanes;          /* batches in flight at once, 1..16 */
    int32_t max_batch;      /* most requests in one batch, 1..65536 */
    int32_t global_slots;   /* global-tier searches each lane runs at once, 1..256 */
    int64_t hbm_budget;     /* bytes of estimated device footprint in flight, > 0 */
    int32_t heavy_lane;     /* 1 (with lanes >= 2): requests of large estimated search work run one
                               at a time on the last lane, the other lanes take the rest (and the
                               first heavy request while the last lane is busy and no light request
                               waits); 0: every lane takes requests in arrival order */
    int32_t reserved;
} rn_server_config;

typedef struct rn_server_stats {
    int64_t submitted;      /* requests accepted */
    int64_t completed;      /* requests answered (including argument errors) */
    int64_t batches;        /* batches launched */
    int64_t reruns;         /* batches re-run with larger buffers */
    int64_t peak_budget;    /* largest estimated footprint in flight, bytes */
    int64_t device_bytes;   /* largest device memory held by the lanes (all their buffers), bytes */
    int32_t max_in_flight;  /* most requests in flight at once */
    int32_t max_lanes_busy; /* most lanes busy at once */
    int32_t max_batch_seen; /* largest batch launched */
    int32_t budget_waits;   /* requests held back at least once because they did not fit the budget */
} rn_server_stats;

/* Start a server on graph cfg->graph of g (device work runs on lane streams
 * the server creates).  RN_ERR_ARG on a bad configuration, RN_ERR_BUSY if the
 * handle is in use. */
rn_status rn_server_create(rn_graph *g, const rn_server_config *cfg, rn_server **out);

/*
 * Submit a request; returns at once with its id.  R, S are HOST arrays (copied
 * before the call returns) with the rules of rn_dist_join; k = 0 asks for the
 * theta-join, k >= 1 for the k closest pairs within theta (theta = 2^32 - 2:
 * unbounded).  RN_ERR_ARG for counts, k or theta out of range; invalid ids,
 * duplicates or overlaps are reported by rn_server_wait.
 */
rn_status rn_server_submit(rn_server *s, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, uint32_t theta,
                           int32_t k, int64_t *id);

/*
 * Wait for request id, then copy its pairs (sorted by (dist, u, v)) to the
 * HOST buffer out[0 .. *n_out) and release the request.  latency_ms (may be
 * NULL) receives the time from submission to the result reaching the host.
 * RN_ERR_CAPACITY (request kept, *n_out set) if cap is too small; the
 * request's own error (RN_ERR_ARG for invalid node sets, ...) otherwise.
 */
rn_status rn_server_wait(rn_server *s, int64_t id, rn_pair *out, int64_t cap, int64_t *n_out, double *latency_ms);

rn_status rn_server_get_stats(rn_server *s, rn_server_stats *out);

/* Finish every submitted request, stop the server and free it (NULL accepted). */
void rn_server_free(rn_server *s);

/*
 * rn_dist_join_noalloc -- rn_dist_join for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * rn_dist_join, but every device buffer of the call (call state, staging,
 * source lists, record buffers and, when a search needs them, global-tier
 * slots) is carved out of one static device array of
 * RN_NOALLOC_SCRATCH_BYTES per GPU, held by the library from its first use
 * on that GPU until the process ends; nothing is allocated per call.  Limits:
 * the call's records must fit that array (RN_ERR_NOMEM otherwise, with a
 * message giving both counts: about 4 million records), and a search that
 * outgrows every on-chip table runs with at most 8 global-tier slots, or fails
 * with RN_ERR_NOMEM when one slot does not fit.  Every call on a GPU uses that
 * GPU's array: calls that overlap on one GPU (from several threads or
 * streams) race and must not be issued.  The call waits for its work before
 * returning, as rn_dist_join does.
 */
#define RN_NOALLOC_SCRATCH_BYTES (128u << 20)
rn_status rn_dist_join_noalloc(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                               uint32_t theta, rn_pair *out, int64_t cap, int64_t *n_out, void *stream);

/* Per-call statistics of the most recent join on a handle. */
typedef struct rn_stats {
    float stage_ms;      /* validation and source staging kernels */
    float relax_ms;      /* bucketed relaxation + pair emission, first attempt */
    float retry_ms;      /* re-runs of sources whose search outgrew the first table */
    float select_ms;     /* k-closest pairs: bound seeding and final selection */
    float sort_ms;       /* canonical (dist, u, v) ordering and copy-out */
    float total_ms;      /* all device work of the call */
    int64_t pairs;       /* pairs produced (before the k cut for k-closest pairs) */
    int64_t arcs;        /* work count: out-arcs of every settled (source, vertex) */
    int64_t settled;     /* work count: settled (source, vertex) pairs */
    int32_t retried;     /* sources re-run after outgrowing the first on-chip table */
    int32_t global_searches; /* sources that outgrew every on-chip table (global-memory tier) */
    int32_t relax_launches; /* relaxation launches (on-chip tiers + the global tier) */
} rn_stats;

/* Profiling flags for rn_set_profiling. */
#define RN_PROFILE_TIMES 1  /* HIP-event timing of each stage (times are 0 otherwise) */
#define RN_PROFILE_WORK  2  /* count arcs / settled vertices (costs extra loads) */

/*
 * Select profiling of the joins on this handle (a bitwise OR of RN_PROFILE_*,
 * 0 = off); rn_last_stats then reports per-stage device times in ms and, with
 * RN_PROFILE_WORK, the work counts.  The arc count is the number of arcs a
 * work-efficient search scans: the sum over sources u of the out-degrees of
 * all vertices within the bound of u.
 */
rn_status rn_set_profiling(rn_graph *g, int32_t on);
rn_status rn_last_stats(const rn_graph *g, rn_stats *out);

/* Message for the calling thread's most recent failure ("" if none). */
const char *rn_last_error(void);

/* Library version string. */
const char *rn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RN_H */
