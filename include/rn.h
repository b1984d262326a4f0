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
 */
rn_status rn_graph_load(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col,
                        const uint32_t *w, rn_graph **out);

/* Free a handle and all its device memory.  NULL is accepted. */
void rn_graph_free(rn_graph *g);

/* Number of vertices / arcs of a loaded graph (0 for NULL). */
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
 * rn_partition -- partition a loaded graph (as rn_partition_host) and keep the
 * leaf-by-leaf vertex order in the handle.  Later joins visit their sources in
 * that order, so sources of one leaf run next to each other on the device
 * (well-separated regions, Section 3).  Join results never depend on it.
 *   part_out  host int32[V] or NULL, as in rn_partition_host
 */
rn_status rn_partition(rn_graph *g, float alpha, int32_t max_leaf, int32_t *part_out);

/*
 * rn_dist_join -- the theta-join.
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
 * rn_kcp_join -- the k-closest-pairs join.
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
 *                (frontier-synchronous relaxation).  Default chosen at load.
 *   hash_log2    log2 of the per-source LDS table size tried first (8..14);
 *                sources whose search outgrows it are re-run with larger ones.
 * Pass a negative value to keep a knob's current setting.
 */
rn_status rn_set_tuning(rn_graph *g, int64_t delta, int32_t hash_log2);
rn_status rn_get_tuning(const rn_graph *g, uint32_t *delta, int32_t *hash_log2);

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
