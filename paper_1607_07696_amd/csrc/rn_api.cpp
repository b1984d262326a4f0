// rn_api.cpp -- host side of the C ABI declared in include/rn.h.
//
// Owns graph residency (rn_graph_load), query buffers, argument checks, the
// launch sequence of a join and the read-back of its control block.  All
// device work of a call is enqueued on the caller's stream; the call waits for
// it once, at the end, to report the result count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rn.h"
#include "rn_internal.h"
#include "rn_partition.h"

using namespace rn;

namespace {

thread_local std::string t_err;

rn_status fail(rn_status st, const std::string &msg) {
    t_err = msg;
    return st;
}

rn_status hip_fail(hipError_t e, const char *what) {
    return fail(RN_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define RN_HIP(call, what)                                  \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return hip_fail(_e, what);    \
    } while (0)

template <typename T>
hipError_t dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Stage timing events (used when profiling is on).
enum { EV_START, EV_STAGED, EV_TIER0, EV_RELAXED, EV_SELECTED, EV_DONE, EV_COUNT };

}  // namespace

struct rn_graph {
    int device = 0;
    int32_t V = 0;
    int64_t A = 0;
    std::vector<int32_t> row_ptr, col;
    std::vector<uint32_t> w;
    uint32_t w_min = 0, w_max = 0;

    int32_t *d_row_ptr = nullptr;
    ArcRec *d_arcs = nullptr;
    int32_t *d_rank = nullptr;    // vertex -> rank in the source order (nullptr = identity)
    int32_t *d_order = nullptr;   // rank -> vertex

    uint32_t delta = 0;
    int hash_log2 = 11;

    // query buffers (grown on demand)
    uint32_t *d_qblock = nullptr;  // QueryCtl | S bitmap | R bitmap | sort histograms, cleared as one
    size_t qblock_words = 0;
    int32_t *d_src = nullptr;
    uint32_t *d_ovf[kTiers] = {};
    size_t src_cap = 0;
    rn_pair *d_pairs[2] = {};
    unsigned long long pair_cap = 0;
    uint32_t *d_stage = nullptr;   // source-listing block sums
    uint32_t *d_gslots = nullptr;  // global-memory tier state (global_slot_words(V) per slot)
    uint32_t n_gslots = 0;
    QueryCtl *h_ctl = nullptr;     // pinned read-back of the control block

    std::atomic<int> busy{0};
    bool profiling = false;
    bool count_work = false;
    hipEvent_t ev[EV_COUNT] = {};
    rn_stats stats{};

    // bitmap sizes rounded to 256-byte multiples keep every region 16-byte aligned
    size_t bitmap_words() const { return ((static_cast<size_t>(V) + 31) / 32 + 63) / 64 * 64; }
    size_t ctl_words() const { return (sizeof(QueryCtl) + 255) / 256 * 64; }
    QueryCtl *d_ctl() const { return reinterpret_cast<QueryCtl *>(d_qblock); }
    uint32_t *d_sbits() const { return d_qblock + ctl_words(); }
    uint32_t *d_rbits() const { return d_qblock + ctl_words() + bitmap_words(); }
    uint32_t *d_hist() const { return d_qblock + ctl_words() + 2 * bitmap_words(); }
    uint32_t *d_seed_hist() const { return d_hist() + sort_hist_words(); }
    uint32_t *d_cand_hist() const { return d_seed_hist() + kDistBins; }
};

namespace {

struct BusyGuard {
    rn_graph *g;
    bool ok;
    explicit BusyGuard(rn_graph *gg) : g(gg) {
        int expect = 0;
        ok = g->busy.compare_exchange_strong(expect, 1);
    }
    ~BusyGuard() {
        if (ok) g->busy.store(0);
    }
};

void release_buffers(rn_graph *g) {
    dev_free(g->d_qblock);
    dev_free(g->d_src);
    for (auto &p : g->d_ovf) dev_free(p);
    dev_free(g->d_pairs[0]);
    dev_free(g->d_pairs[1]);
    dev_free(g->d_stage);
    dev_free(g->d_gslots);
    g->n_gslots = 0;
    g->qblock_words = 0;
    g->src_cap = 0;
    g->pair_cap = 0;
}

rn_status ensure_query_buffers(rn_graph *g, int32_t nR) {
    const size_t qwords = g->ctl_words() + 2 * g->bitmap_words() + sort_hist_words() + 2 * kDistBins;
    if (g->qblock_words < qwords) {
        dev_free(g->d_qblock);
        RN_HIP(dev_alloc(&g->d_qblock, qwords), "allocating query bitmaps");
        g->qblock_words = qwords;
    }
    if (g->src_cap < static_cast<size_t>(nR)) {
        dev_free(g->d_src);
        for (auto &p : g->d_ovf) dev_free(p);
        const size_t cap = std::max<size_t>(static_cast<size_t>(nR), 1024);
        RN_HIP(dev_alloc(&g->d_src, cap), "allocating the source list");
        for (auto &p : g->d_ovf) RN_HIP(dev_alloc(&p, cap), "allocating the re-run lists");
        g->src_cap = cap;
    }
    if (!g->d_stage) RN_HIP(dev_alloc(&g->d_stage, stage_scratch_words(g->V)), "allocating staging scratch");
    if (!g->d_gslots) {
        // up to 64 concurrent global-tier searches, within 8 GiB
        const size_t words = global_slot_words(g->V);
        size_t n = (size_t{8} << 30) / (4 * words);
        n = std::max<size_t>(1, std::min<size_t>(n, 64));
        RN_HIP(dev_alloc(&g->d_gslots, n * words), "allocating global search slots");
        g->n_gslots = static_cast<uint32_t>(n);
        const size_t V = static_cast<size_t>(g->V);
        for (size_t i = 0; i < n; ++i) {
            RN_HIP(launch_fill_u32(g->d_gslots + i * words, V, kInf, nullptr), "clearing search slots");
            RN_HIP(launch_fill_u32(g->d_gslots + i * words + V, (V + 31) / 32, 0u, nullptr),
                   "clearing search slots");
        }
        RN_HIP(hipDeviceSynchronize(), "clearing search slots");
    }
    if (g->pair_cap == 0) {
        const unsigned long long cap = 1ull << 20;
        RN_HIP(dev_alloc(&g->d_pairs[0], cap), "allocating the pair buffer");
        RN_HIP(dev_alloc(&g->d_pairs[1], cap), "allocating the pair buffer");
        g->pair_cap = cap;
    }
    return RN_OK;
}

rn_status grow_pairs(rn_graph *g, unsigned long long need) {
    unsigned long long cap = std::max(need + need / 4, 2 * g->pair_cap);
    dev_free(g->d_pairs[0]);
    dev_free(g->d_pairs[1]);
    g->pair_cap = 0;
    RN_HIP(dev_alloc(&g->d_pairs[0], cap), "growing the pair buffer");
    RN_HIP(dev_alloc(&g->d_pairs[1], cap), "growing the pair buffer");
    g->pair_cap = cap;
    return RN_OK;
}

void record(rn_graph *g, int which, hipStream_t s) {
    if (g->profiling) (void)hipEventRecord(g->ev[which], s);
}

float elapsed(rn_graph *g, int a, int b) {
    float ms = 0.f;
    if (!g->profiling) return 0.f;
    if (hipEventElapsedTime(&ms, g->ev[a], g->ev[b]) != hipSuccess) return 0.f;
    return ms;
}

// On-chip table tiers tried in order: the handle's first choice (a small table
// for k-closest pairs, whose searches are usually cut short by the bound),
// then larger ones; the global-memory tier follows them.
int tier_list(const rn_graph *g, bool kcp, int *hb) {
    int n = 0;
    const int first = kcp ? 8 : g->hash_log2;
    const int cand[kLdsTiers] = {first, std::min(std::max(first + 3, g->hash_log2), 14), 14};
    for (int c : cand)
        if (n == 0 || c > hb[n - 1]) hb[n++] = c;
    return n;
}

rn_status check_sets(const rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                     int64_t *n_out) {
    if (!n_out) return fail(RN_ERR_ARG, "n_out is NULL");
    *n_out = 0;
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (nR < 1 || nS < 1) return fail(RN_ERR_ARG, "R and S must each hold at least one vertex");
    if (!R || !S) return fail(RN_ERR_ARG, "R or S is NULL");
    if (static_cast<int64_t>(nR) + nS > static_cast<int64_t>(g->V))
        return fail(RN_ERR_ARG, "R and S together exceed the vertex count (they must be disjoint)");
    return RN_OK;
}

std::string describe_err(uint32_t err) {
    std::string m = "invalid node sets:";
    if (err & kErrRange) m += " id outside [0, V);";
    if (err & kErrDupR) m += " duplicate in R;";
    if (err & kErrDupS) m += " duplicate in S;";
    if (err & kErrOverlap) m += " R and S overlap;";
    return m;
}

// The shared launch sequence of both joins.  `bound` is theta (theta-join) or
// the largest distance a k-closest-pairs answer may hold.
rn_status run_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                   uint32_t bound, bool kcp, int32_t k, rn_pair *out, int64_t cap, int64_t *n_out,
                   hipStream_t stream);

}  // namespace

extern "C" {

const char *rn_last_error(void) { return t_err.c_str(); }

const char *rn_version(void) { return "rn 0.1 (gfx950)"; }

rn_status rn_graph_load(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col,
                        const uint32_t *w, rn_graph **out) {
    if (!out) return fail(RN_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (V < 1 || V >= 0x7FFFFFFF) return fail(RN_ERR_ARG, "V must be in [1, 2^31 - 2]");
    if (A < 0 || A >= 0x7FFFFFFFLL) return fail(RN_ERR_ARG, "A must be in [0, 2^31 - 1]");
    if (!row_ptr || (A > 0 && (!col || !w))) return fail(RN_ERR_ARG, "CSR array is NULL");
    if (row_ptr[0] != 0 || static_cast<int64_t>(row_ptr[V]) != A)
        return fail(RN_ERR_ARG, "row_ptr must start at 0 and end at A");
    for (int32_t x = 0; x < V; ++x)
        if (row_ptr[x + 1] < row_ptr[x]) return fail(RN_ERR_ARG, "row_ptr must be non-decreasing");
    for (int64_t a = 0; a < A; ++a)
        if (col[a] < 0 || col[a] >= V) return fail(RN_ERR_ARG, "col entry outside [0, V)");

    rn_graph *g = new (std::nothrow) rn_graph();
    if (!g) return fail(RN_ERR_NOMEM, "allocating the handle");
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "no HIP device");
    }
    g->V = V;
    g->A = A;
    try {
        g->row_ptr.assign(row_ptr, row_ptr + V + 1);
        g->col.assign(col, col + A);
        g->w.assign(w, w + A);
    } catch (...) {
        delete g;
        return fail(RN_ERR_NOMEM, "copying the CSR");
    }
    g->w_min = A ? *std::min_element(g->w.begin(), g->w.end()) : 0;
    g->w_max = A ? *std::max_element(g->w.begin(), g->w.end()) : 0;

    std::vector<ArcRec> arcs(static_cast<size_t>(A));
    for (int64_t a = 0; a < A; ++a) {
        const int32_t y = col[a];
        arcs[a] = ArcRec{y, w[a], row_ptr[y], row_ptr[y + 1]};
    }
    rn_status st = RN_OK;
    if ((e = dev_alloc(&g->d_row_ptr, static_cast<size_t>(V) + 1)) != hipSuccess ||
        (e = dev_alloc(&g->d_arcs, static_cast<size_t>(A))) != hipSuccess ||
        (e = hipMemcpy(g->d_row_ptr, row_ptr, (static_cast<size_t>(V) + 1) * sizeof(int32_t),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (A > 0 && (e = hipMemcpy(g->d_arcs, arcs.data(), static_cast<size_t>(A) * sizeof(ArcRec),
                                 hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipHostMalloc(reinterpret_cast<void **>(&g->h_ctl), sizeof(QueryCtl), 0)) != hipSuccess) {
        st = hip_fail(e, "uploading the graph");
    }
    for (int i = 0; st == RN_OK && i < EV_COUNT; ++i)
        if ((e = hipEventCreate(&g->ev[i])) != hipSuccess) st = hip_fail(e, "creating events");
    if (st != RN_OK) {
        rn_graph_free(g);
        return st;
    }
    g->delta = 0;
    g->hash_log2 = 11;
    *out = g;
    return RN_OK;
}

void rn_graph_free(rn_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    release_buffers(g);
    dev_free(g->d_row_ptr);
    dev_free(g->d_arcs);
    dev_free(g->d_rank);
    dev_free(g->d_order);
    if (g->h_ctl) (void)hipHostFree(g->h_ctl);
    for (auto &ev : g->ev)
        if (ev) (void)hipEventDestroy(ev);
    delete g;
}

int32_t rn_graph_num_vertices(const rn_graph *g) { return g ? g->V : 0; }
int64_t rn_graph_num_arcs(const rn_graph *g) { return g ? g->A : 0; }

rn_status rn_partition_host(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col,
                            const uint32_t *w, float alpha, int32_t max_leaf, int32_t *part_out,
                            int32_t *order_out) {
    if (V < 1 || A < 0 || !row_ptr || (A > 0 && (!col || !w)))
        return fail(RN_ERR_ARG, "malformed CSR");
    if (row_ptr[0] != 0 || static_cast<int64_t>(row_ptr[V]) != A)
        return fail(RN_ERR_ARG, "row_ptr must start at 0 and end at A");
    for (int32_t x = 0; x < V; ++x)
        if (row_ptr[x + 1] < row_ptr[x]) return fail(RN_ERR_ARG, "row_ptr must be non-decreasing");
    for (int64_t a = 0; a < A; ++a)
        if (col[a] < 0 || col[a] >= V) return fail(RN_ERR_ARG, "col entry outside [0, V)");
    if (!(alpha >= 0.f && alpha <= 1.f)) return fail(RN_ERR_ARG, "alpha must be in [0, 1]");
    if (max_leaf < 1) return fail(RN_ERR_ARG, "max_leaf must be >= 1");
    std::vector<int32_t> part, order;
    std::string msg;
    if (!partition_graph(V, row_ptr, col, w, alpha, max_leaf, part, order, msg))
        return fail(RN_ERR_NOMEM, msg);
    if (part_out) std::memcpy(part_out, part.data(), static_cast<size_t>(V) * sizeof(int32_t));
    if (order_out) std::memcpy(order_out, order.data(), static_cast<size_t>(V) * sizeof(int32_t));
    return RN_OK;
}

rn_status rn_partition(rn_graph *g, float alpha, int32_t max_leaf, int32_t *part_out) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    std::vector<int32_t> order(static_cast<size_t>(g->V));
    rn_status st = rn_partition_host(g->V, g->A, g->row_ptr.data(), g->col.data(), g->w.data(), alpha,
                                     max_leaf, part_out, order.data());
    if (st != RN_OK) return st;
    std::vector<int32_t> rank(static_cast<size_t>(g->V));
    for (int32_t r = 0; r < g->V; ++r) rank[order[r]] = r;
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    if (!g->d_rank) RN_HIP(dev_alloc(&g->d_rank, static_cast<size_t>(g->V)), "allocating ranks");
    if (!g->d_order) RN_HIP(dev_alloc(&g->d_order, static_cast<size_t>(g->V)), "allocating ranks");
    RN_HIP(hipMemcpy(g->d_rank, rank.data(), rank.size() * sizeof(int32_t), hipMemcpyHostToDevice),
           "uploading ranks");
    RN_HIP(hipMemcpy(g->d_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice),
           "uploading ranks");
    return RN_OK;
}

rn_status rn_set_tuning(rn_graph *g, int64_t delta, int32_t hash_log2) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (delta > static_cast<int64_t>(kMaxDist)) return fail(RN_ERR_ARG, "delta out of range");
    if (hash_log2 >= 0 && !join_tier_supported(hash_log2))
        return fail(RN_ERR_ARG, "hash_log2 must be in [8, 14]");
    if (delta >= 0) g->delta = static_cast<uint32_t>(delta);
    if (hash_log2 >= 0) g->hash_log2 = hash_log2;
    return RN_OK;
}

rn_status rn_get_tuning(const rn_graph *g, uint32_t *delta, int32_t *hash_log2) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (delta) *delta = g->delta;
    if (hash_log2) *hash_log2 = g->hash_log2;
    return RN_OK;
}

rn_status rn_set_profiling(rn_graph *g, int32_t on) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    g->profiling = (on & RN_PROFILE_TIMES) != 0;
    g->count_work = (on & RN_PROFILE_WORK) != 0;
    return RN_OK;
}

rn_status rn_last_stats(const rn_graph *g, rn_stats *out) {
    if (!g || !out) return fail(RN_ERR_ARG, "NULL argument");
    *out = g->stats;
    return RN_OK;
}

rn_status rn_dist_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                       uint32_t theta, rn_pair *out, int64_t cap, int64_t *n_out, void *stream) {
    rn_status st = check_sets(g, R, nR, S, nS, n_out);
    if (st != RN_OK) return st;
    if (theta > kMaxDist) return fail(RN_ERR_ARG, "theta must be <= 2^32 - 2");
    if (cap < 0 || (cap > 0 && !out)) return fail(RN_ERR_ARG, "bad output buffer");
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    return run_join(g, R, nR, S, nS, theta, false, 0, out, cap, n_out,
                    reinterpret_cast<hipStream_t>(stream));
}

rn_status rn_kcp_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                      int32_t k, rn_pair *out, int64_t cap, int64_t *n_out, void *stream) {
    rn_status st = check_sets(g, R, nR, S, nS, n_out);
    if (st != RN_OK) return st;
    if (k < 1 || k > (1 << 24)) return fail(RN_ERR_ARG, "k must be in [1, 2^24]");
    if (cap < 0 || (cap > 0 && !out)) return fail(RN_ERR_ARG, "bad output buffer");
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    return run_join(g, R, nR, S, nS, kMaxDist, true, k, out, cap, n_out,
                    reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

rn_status run_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                   uint32_t bound, bool kcp, int32_t k, rn_pair *out, int64_t cap, int64_t *n_out,
                   hipStream_t stream) {
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    rn_status st = ensure_query_buffers(g, nR);
    if (st != RN_OK) return st;
    int hb[kLdsTiers];
    const int nlds = tier_list(g, kcp, hb);
    const int ntiers = nlds + 1;
    QueryCtl *ctl = g->d_ctl();
    g->stats = rn_stats{};

    for (int attempt = 0; attempt < 3; ++attempt) {
        record(g, EV_START, stream);
        RN_HIP(launch_fill_u32(g->d_qblock, g->qblock_words, 0u, stream), "clearing query state");
        RN_HIP(launch_stage(R, nR, S, nS, g->V, g->d_rank, g->d_order, g->d_rbits(), g->d_sbits(),
                            g->d_src, ctl, g->d_stage, stream),
               "staging the query");
        record(g, EV_STAGED, stream);
        if (kcp)
            RN_HIP(launch_kcp_seed(g->d_src, &ctl->nsrc, static_cast<uint32_t>(nR), g->d_row_ptr, g->d_arcs,
                                   g->d_sbits(), g->d_seed_hist(), static_cast<uint32_t>(k), ctl, stream),
                   "seeding the k-closest-pairs bound");
        for (int t = 0; t < ntiers; ++t) {
            JoinArgs a;
            a.row_ptr = g->d_row_ptr;
            a.arcs = g->d_arcs;
            a.sbits = g->d_sbits();
            a.src = t == 0 ? g->d_src : reinterpret_cast<const int32_t *>(g->d_ovf[t - 1]);
            a.nsrc = t == 0 ? &ctl->nsrc : &ctl->novf[t - 1];
            a.ctl = ctl;
            a.pairs = g->d_pairs[0];
            a.pair_cap = g->pair_cap;
            a.ovf = g->d_ovf[t];
            a.novf = &ctl->novf[t];
            a.theta = bound;
            a.delta = g->delta;
            a.kcp = kcp ? 1 : 0;
            a.count_work = g->count_work ? 1 : 0;
            a.k = static_cast<uint32_t>(k);
            a.cand_hist = g->d_cand_hist();
            if (t < nlds)
                RN_HIP(launch_join(a, hb[t], static_cast<uint32_t>(nR), stream), "launching the relaxation");
            else
                RN_HIP(launch_join_global(a, g->d_gslots, g->n_gslots, g->V, static_cast<uint32_t>(nR),
                                          stream),
                       "launching the global relaxation");
            if (t == 0) record(g, EV_TIER0, stream);
        }
        record(g, EV_RELAXED, stream);
        if (!kcp) {
            record(g, EV_SELECTED, stream);
            RN_HIP(launch_sort_to_out(g->d_pairs[0], g->d_pairs[1], &ctl->npairs, g->pair_cap, bound, g->V,
                                      g->d_hist(), out, static_cast<unsigned long long>(cap), ~0ull, ctl,
                                      ntiers - 1, stream),
                   "sorting pairs");
        } else {
            // the final bound fixes the sort key width: read it back first
            RN_HIP(hipMemcpyAsync(g->h_ctl, ctl, sizeof(QueryCtl), hipMemcpyDeviceToHost, stream),
                   "reading the query status");
            RN_HIP(hipStreamSynchronize(stream), "waiting for the searches");
            const QueryCtl c = *g->h_ctl;
            if (c.err) return fail(RN_ERR_ARG, describe_err(c.err));
            if (c.npairs > g->pair_cap) {
                st = grow_pairs(g, c.npairs);
                if (st != RN_OK) return st;
                continue;
            }
            RN_HIP(launch_kcp_filter(g->d_pairs[0], g->pair_cap, g->d_pairs[1], ctl, stream),
                   "filtering candidates");
            record(g, EV_SELECTED, stream);
            RN_HIP(launch_sort_to_out(g->d_pairs[1], g->d_pairs[0], &ctl->nsel, g->pair_cap, c.theta, g->V,
                                      g->d_hist(), out, static_cast<unsigned long long>(cap),
                                      static_cast<unsigned long long>(k), ctl, ntiers - 1, stream),
                   "sorting pairs");
        }
        record(g, EV_DONE, stream);
        RN_HIP(hipMemcpyAsync(g->h_ctl, ctl, sizeof(QueryCtl), hipMemcpyDeviceToHost, stream),
               "reading the query status");
        RN_HIP(hipStreamSynchronize(stream), "waiting for the query");
        const QueryCtl c = *g->h_ctl;
        if (c.err) return fail(RN_ERR_ARG, describe_err(c.err));
        if (c.novf[ntiers - 1]) return fail(RN_ERR_DEVICE, "global search tier overflowed");
        if (c.npairs > g->pair_cap) {
            st = grow_pairs(g, c.npairs);
            if (st != RN_OK) return st;
            continue;
        }
        g->stats.stage_ms = elapsed(g, EV_START, EV_STAGED);
        g->stats.relax_ms = elapsed(g, EV_STAGED, EV_TIER0);
        g->stats.retry_ms = elapsed(g, EV_TIER0, EV_RELAXED);
        g->stats.select_ms = elapsed(g, EV_RELAXED, EV_SELECTED);
        g->stats.sort_ms = elapsed(g, EV_SELECTED, EV_DONE);
        g->stats.total_ms = elapsed(g, EV_START, EV_DONE);
        g->stats.pairs = static_cast<int64_t>(c.npairs);
        g->stats.arcs = static_cast<int64_t>(c.arcs);
        g->stats.settled = static_cast<int64_t>(c.settled);
        g->stats.retried = static_cast<int32_t>(c.novf[0]);
        g->stats.global_searches = static_cast<int32_t>(c.novf[nlds - 1]);
        g->stats.relax_launches = ntiers;
        const unsigned long long n =
            kcp ? std::min<unsigned long long>(c.nsel, static_cast<unsigned long long>(k)) : c.npairs;
        *n_out = static_cast<int64_t>(n);
        if (n > static_cast<unsigned long long>(cap)) return fail(RN_ERR_CAPACITY, "output buffer too small");
        return RN_OK;
    }
    return fail(RN_ERR_NOMEM, "pair buffer did not settle");
}

}  // namespace
