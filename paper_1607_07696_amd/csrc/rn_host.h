// rn_host.h -- host-side call machinery shared by the C ABI (rn_api.cpp) and
// the request server (rn_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <vector>

#include "rn.h"
#include "rn_internal.h"

struct rn_graph;

namespace rn {
namespace host {

// Set the calling thread's error message (rn_last_error) and return st.
rn_status fail(rn_status st, const std::string &msg);
rn_status hip_fail(hipError_t e, const char *what);
const std::string &last_error();

#define RN_HIP(call, what)                                  \
    do {                                                    \
        hipError_t _e = (call);                             \
        if (_e != hipSuccess) return hip_fail(_e, what);    \
    } while (0)

#define RN_TRY(call)                          \
    do {                                      \
        rn_status _s = (call);                \
        if (_s != RN_OK) return _s;           \
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

template <typename T>
void host_free(T *&p) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
}

// Stage timing events (used when profiling is on).
enum { EV_START, EV_STAGED, EV_TIER0, EV_RELAXED, EV_SELECTED, EV_DONE, EV_COUNT };

constexpr int kSide = 2 * (kMaxHB - kMinHB + 1) - 1;   // side streams: one per first-tier launch beyond the first
constexpr unsigned long long kRecCapMax = 1ull << 31;

inline size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

inline uint32_t bitlen(uint64_t x) {
    uint32_t b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

// Device and pinned host buffers of calls, with the global-tier search slots;
// a handle owns one for its eager calls, every plan and every server lane its own.
struct Workspace {
    uint32_t *d_block = nullptr;    // CallCtl | QueryState[nq] | S bitmaps | rank bitmaps | histograms | sort
    size_t block_words = 0;
    uint8_t *d_desc = nullptr;      // QueryDesc[nq] | ebase[nq+1] | rbase[nq+1] | perm[nq]
    size_t desc_bytes = 0;
    uint8_t *h_desc = nullptr;      // pinned staging of the same
    size_t h_desc_bytes = 0;
    uint8_t *h_state = nullptr;     // pinned read-back of CallCtl | QueryState[nq], mapped:
    uint32_t *d_state_map = nullptr;  //   its device address, written by the call's last kernel
    size_t h_state_bytes = 0;
    uint32_t *d_stage = nullptr;
    size_t stage_words = 0;
    int32_t *d_src = nullptr;
    uint32_t *d_srcq = nullptr;
    int32_t *d_list[kLists] = {};
    uint32_t *d_listq[kLists] = {};
    size_t src_cap = 0;
    Rec *d_recs[2] = {};
    unsigned long long rec_cap = 0;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSide] = {};
    hipEvent_t ev[EV_COUNT] = {};
    uint32_t *d_gslots = nullptr;   // global_slot_words(Vmax) words per slot, allocated when
    uint32_t n_gslots = 0;          //   a call first sends a search to the global tier
    uint32_t gslot_cap = 256;       // most slots this workspace allocates

    void release() {
        dev_free(d_gslots);
        n_gslots = 0;
        dev_free(d_block);
        dev_free(d_desc);
        host_free(h_desc);
        host_free(h_state);
        d_state_map = nullptr;
        dev_free(d_stage);
        dev_free(d_src);
        dev_free(d_srcq);
        for (int i = 0; i < kLists; ++i) {
            dev_free(d_list[i]);
            dev_free(d_listq[i]);
        }
        dev_free(d_recs[0]);
        dev_free(d_recs[1]);
        block_words = desc_bytes = h_desc_bytes = h_state_bytes = stage_words = src_cap = 0;
        rec_cap = 0;
        for (auto &s : side)
            if (s) (void)hipStreamDestroy(s), s = nullptr;
        if (fork) (void)hipEventDestroy(fork), fork = nullptr;
        for (auto &e : join)
            if (e) (void)hipEventDestroy(e), e = nullptr;
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e), e = nullptr;
    }
};

// One group of queries whose searches start with the same table size.
struct Group {
    int hb;
    bool kcp;               // some query of the group asks for k closest pairs
    bool compact;           // its launch uses compact on-chip tables
    int32_t first;          // staging positions [first, end)
    int32_t end;
    uint64_t sources;       // sum of nR
};

// Host-side plan of one call: descriptors, pools and launch shapes.
struct Prepared {
    int32_t nq = 0;
    std::vector<QueryDesc> qd;
    std::vector<unsigned long long> ebase;
    std::vector<uint32_t> rbase;
    std::vector<uint32_t> perm;
    std::vector<Group> groups;
    bool any_kcp = false;
    bool need_list0 = false;
    bool need_list1 = false;
    bool any_global = false;        // a first-tier group runs in the global tier
    uint32_t qb = 0, vb = 1, max_passes = 1;
    uint64_t total_R = 0;
    unsigned long long total_elems = 0;
    // word offsets in the call block
    size_t off_qs = 0, off_sbits = 0, off_rbits = 0, off_hists = 0, off_work = 0, off_sort = 0, block_words = 0;
    size_t zero_words = 0;
    uint32_t sbits_words = 0, rbits_words = 0;
    size_t desc_bytes = 0, off_ebase = 0, off_rbase = 0, off_perm = 0;
    // bucket sort (theta-join calls with few bins); nbins = 0: radix sort
    uint32_t nbins = 0;
    bool small_sort = false;        // k-closest-pairs calls with few candidates: launch_sort_small
    std::vector<uint32_t> binbase;
    size_t off_bins = 0, off_binbase = 0;
};

std::string describe_err(uint32_t err);
// Host-side checks of a batch (status[i] marks the malformed queries).
rn_status check_queries(const rn_graph *g, const rn_query *q, int32_t nq, int32_t *status);
rn_status prepare(const rn_graph *g, const rn_query *q, int32_t nq, Prepared &p);
// Global-tier slots are allocated on demand: a call enqueued while a
// workspace has none skips the global tier, and if any of its searches needed
// it (ctl.nlist[2] > 0) the call is run again once slots exist.  Allocate (once)
// and clear slots for `want` concurrent searches (at most ws.gslot_cap, within
// 48 GiB) for graphs of up to Vmax vertices; the clearing runs on s, which is
// synchronised.
rn_status ensure_gslots(Workspace &ws, int32_t Vmax, uint32_t want, hipStream_t s);
inline size_t gslot_bytes(const Workspace &ws, int32_t Vmax) {
    return static_cast<size_t>(ws.n_gslots) * global_slot_words(Vmax) * 4;
}
rn_status ensure_buffers(Workspace &ws, const Prepared &p);
rn_status grow_recs(Workspace &ws, unsigned long long need);
void fill_host_desc(const Prepared &p, uint8_t *h);
// Enqueue a whole call on s (descriptors already on the device); timed:
// record the profiling events of the handle; shared: the device is shared with
// other streams (no side streams for the first-tier launches, one block per
// source so that other streams' kernels interleave).
rn_status enqueue_call(rn_graph *g, Workspace &ws, const Prepared &p, rn_pair *out, int64_t cap, hipStream_t s,
                       bool timed, bool shared = false);
// After a call whose sort left the output to the radix sort (its state's
// resort: a bucket-sort bin too large to rank, or too many candidates for the
// small sort): enqueue on s the radix sort of the records in recs[1], which
// writes the output.
rn_status enqueue_sort_fallback(const Workspace &ws, const Prepared &p, rn_pair *out, int64_t cap, hipStream_t s);

}  // namespace host
}  // namespace rn


struct rn_graph {
    int device = 0;
    int32_t ngraphs = 0;
    std::vector<int32_t> voff;      // [ngraphs + 1] vertex offsets
    std::vector<int64_t> aoff;      // [ngraphs + 1] arc offsets
    std::vector<uint32_t> w_min;    // per graph (0 when it has no arcs)
    std::vector<uint32_t> gdelta;   // per graph: bucket width of the global-memory tier
    int32_t V = 0;                  // total vertices
    int64_t A = 0;                  // total arcs
    int32_t Vmax = 0;
    std::vector<int32_t> row_ptr, col;   // concatenated, global ids
    std::vector<uint32_t> w;
    bool can_swap = false;          // searches may run from S (reversed arcs available)
    uint32_t rev_rpo = 0;           // row pointer offset of the reversed arcs (0: the graphs are symmetric)
    bool big_deg = false;           // some vertex has 2^16 or more arcs (forward or reversed)

    int32_t *d_row_ptr = nullptr;
    rn::ArcRec *d_arcs = nullptr;
    // The device copy of the graphs is numbered in partition-leaf order once
    // rn_partition has run (identity until then); the two maps, both
    // allocated at load:
    int32_t *d_rank = nullptr;      // global vertex (caller numbering) -> local id in the device copy
    int32_t *d_order = nullptr;     // global vertex of the device copy -> local id in the caller numbering
    uint32_t *d_first = nullptr;    // per arc record: first lightest arc of its (tail, target) pair
    std::vector<char> renumbered;   // per graph: the device copy is in leaf order (else as loaded)

    uint32_t delta = 0;
    int hash_log2 = 11;
    bool hash_auto = true;          // no first table size set: theta-joins size it from theta
    std::vector<double> wmean;      // per graph: mean arc weight
    std::vector<char> varied;       // per graph: at least 16 distinct arc weights

    rn::host::Workspace ws;

    std::atomic<int> busy{0};
    bool profiling = false;
    bool count_work = false;
    rn_stats stats{};
};

struct rn_plan {
    rn_graph *g = nullptr;
    rn::host::Workspace ws;
    std::vector<rn_query> q;
    rn::host::Prepared prep;
    rn_pair *out = nullptr;
    int64_t cap = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace rn {
namespace host {

// Claims a handle for one call (or for a server's lifetime).
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

}  // namespace host
}  // namespace rn
