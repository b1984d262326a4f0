// rn_api.cpp -- host side of the C ABI declared in include/rn.h.
//
// Owns graph residency (one concatenated CSR for all graphs of a handle),
// call buffers, argument checks, the launch sequence of a call and the
// read-back of its control block.  All device work of a call is enqueued on
// the caller's stream; the call waits for it once, at the end, to report the
// result counts.  Single queries are batches of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "rn.h"
#include "rn_host.h"
#include "rn_internal.h"
#include "rn_partition.h"

using namespace rn;
using namespace rn::host;

namespace rn {
namespace host {

namespace {
thread_local std::string t_err;
}

rn_status fail(rn_status st, const std::string &msg) {
    t_err = msg;
    return st;
}

rn_status hip_fail(hipError_t e, const char *what) {
    return fail(RN_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

const std::string &last_error() { return t_err; }

std::string describe_err(uint32_t err) {
    std::string m;
    if (err & kErrRange) m += " id outside [0, V);";
    if (err & kErrDupR) m += " duplicate in R;";
    if (err & kErrDupS) m += " duplicate in S;";
    if (err & kErrOverlap) m += " R and S overlap;";
    return m;
}

// ------------------------------------------------------------------ preparation
rn_status check_queries(const rn_graph *g, const rn_query *q, int32_t nq, int32_t *status) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (!q || nq < 1 || nq > kMaxQueries) return fail(RN_ERR_ARG, "need 1 to 65536 queries");
    int bad = -1;
    std::string why;
    uint64_t total_R = 0;
    for (int32_t i = 0; i < nq; ++i) {
        const rn_query &x = q[i];
        const char *m = nullptr;
        if (x.graph < 0 || x.graph >= g->ngraphs) m = "graph index out of range";
        else if (x.nR < 1 || x.nS < 1) m = "R and S must each hold at least one vertex";
        else if (!x.R || !x.S) m = "R or S is NULL";
        else if (static_cast<int64_t>(x.nR) + x.nS > g->voff[x.graph + 1] - g->voff[x.graph])
            m = "R and S together exceed the vertex count (they must be disjoint)";
        else if (x.k < 0 || x.k > (1 << 24)) m = "k must be 0 (theta-join) or in [1, 2^24]";
        else if (x.theta > kMaxDist) m = "theta must be <= 2^32 - 2";
        else if (x.hash_log2 != 0 && x.hash_log2 != kGlobalHB && !join_tier_supported(x.hash_log2))
            m = "hash_log2 must be 0, in [8, 14] or RN_TABLE_GLOBAL";
        else if (x.flags & ~RN_QUERY_FORWARD) m = "unknown query flags";
        if (status) status[i] = m ? RN_ERR_ARG : RN_OK;
        if (m && bad < 0) {
            bad = i;
            why = m;
        }
        total_R += static_cast<uint64_t>(std::max(x.nR, 0));
    }
    if (bad >= 0) return fail(RN_ERR_ARG, "query " + std::to_string(bad) + ": " + why);
    if (total_R >= 0x7FFFFFFFull) return fail(RN_ERR_ARG, "the queries' R sets together exceed 2^31 - 2 sources");
    return RN_OK;
}

// First on-chip table of a theta-join when the caller set none: the handle's
// size, raised to hold 1.3x the expected ball (a planar road graph holds
// about 2 (theta / mean arc weight)^2 vertices within theta; a table is
// filled to 3/4).  Larger balls would overflow the small table and re-run.
int first_table(const rn_graph *g, int32_t graph, uint32_t theta) {
    if (!g->hash_auto) return g->hash_log2;
    const double r = static_cast<double>(theta) / std::max(1.0, g->wmean[graph]);
    const double need = 1.3 * 2.0 * r * r / 0.75;
    int hb = g->hash_log2;
    while (hb < kMaxHB && static_cast<double>(1u << hb) < need) ++hb;
    return hb;
}

// Queries whose searches are sure to outgrow the largest on-chip table go to
// the global tier from the start instead of failing through every tier: a
// theta-join whose expected ball (as first_table estimates it, capped at the
// graph) needs more than twice the largest table, and a k-closest-pairs query
// asking for at least half of its pairs on a graph of 2^16 vertices or more
// (its searches then reach past the median R-S distance, a large share of
// the graph).
bool sure_global(const rn_graph *g, const rn_query &x) {
    if (!g->hash_auto) return false;
    const double V = static_cast<double>(g->voff[x.graph + 1] - g->voff[x.graph]);
    const double r = static_cast<double>(x.theta) / std::max(1.0, g->wmean[x.graph]);
    const double ball = std::min(V, 2.0 * r * r);
    const double cap = 0.75 * static_cast<double>(1u << kMaxHB);
    if (x.k == 0) return 1.3 * ball > 2.0 * cap;
    const double pairs = static_cast<double>(x.nR) * static_cast<double>(x.nS);
    return 2.0 * static_cast<double>(x.k) >= pairs && V >= 65536.0 && ball > 2.0 * cap;
}

// The on-chip search with delta = 0 takes the oldest pending vertices in
// steps of 64; a vertex more than the slack above the least distance of its
// step waits for a later one, since its distance is likely to improve
// first.  1.5 mean arc weights: on road graphs this cuts the arcs relaxed
// per search by a fifth (at theta of about 23 mean weights) without adding
// steps; a much smaller slack adds steps, a much larger one defers nothing.
uint32_t ring_slack(double wmean) {
    const double s = 1.5 * wmean;
    return s >= 2147483647.0 ? 0x7FFFFFFFu : static_cast<uint32_t>(s + 0.5);
}

rn_status prepare(const rn_graph *g, const rn_query *q, int32_t nq, Prepared &p) {
    // reset in place: the vectors keep their capacity, so a Prepared reused for
    // calls of the same shape allocates nothing after its first call
    auto qd = std::move(p.qd);
    auto ebase = std::move(p.ebase);
    auto rbase = std::move(p.rbase);
    auto perm = std::move(p.perm);
    auto groups = std::move(p.groups);
    auto binbase = std::move(p.binbase);
    p = Prepared{};
    p.qd = std::move(qd);
    p.ebase = std::move(ebase);
    p.rbase = std::move(rbase);
    p.perm = std::move(perm);
    p.groups = std::move(groups);
    p.binbase = std::move(binbase);
    p.groups.clear();
    p.nq = nq;
    p.qd.resize(nq);
    p.ebase.assign(nq + 1, 0);
    p.rbase.assign(nq + 1, 0);
    p.perm.resize(nq);
    std::vector<int> hb(nq);
    uint32_t dmax = 0;
    for (int32_t i = 0; i < nq; ++i) {
        const rn_query &x = q[i];
        hb[i] = x.hash_log2 ? x.hash_log2
                            : (sure_global(g, x) ? kGlobalHB : (x.k ? kMinHB : first_table(g, x.graph, x.theta)));
        p.any_kcp |= x.k > 0;
        dmax = std::max(dmax, x.theta);
        p.total_R += static_cast<uint64_t>(std::max(x.nR, 0));
    }
    // staging order: grouped by first table size and kind, query order within a group
    for (int32_t i = 0; i < nq; ++i) p.perm[i] = static_cast<uint32_t>(i);
    // (every query searched in the global tier from the start forms one group:
    // a launch of that tier uses every slot, so two could not run side by side)
    auto kcp_part = [&](uint32_t i) { return hb[i] != kGlobalHB && q[i].k > 0; };
    auto key = [&](uint32_t i) { return 2 * hb[i] + (kcp_part(i) ? 1 : 0); };
    std::stable_sort(p.perm.begin(), p.perm.end(), [&](uint32_t a, uint32_t b) { return key(a) < key(b); });
    uint64_t sw = 0, rw = 0;
    uint32_t nkcp = 0;
    for (int32_t s = 0; s < nq; ++s) {
        const uint32_t i = p.perm[s];
        const rn_query &x = q[i];
        const int32_t V = g->voff[x.graph + 1] - g->voff[x.graph];
        const uint32_t words = static_cast<uint32_t>((static_cast<int64_t>(V) + 31) / 32);
        QueryDesc &d = p.qd[i];
        std::memset(&d, 0, sizeof(d));
        // search from the smaller side: with fewer vertices in S than in R the
        // searches run from S over the reversed arcs (pairs are turned back on emission)
        const bool swap = g->can_swap && !(x.flags & RN_QUERY_FORWARD) && x.nS < x.nR;
        d.R = swap ? x.S : x.R;
        d.S = swap ? x.R : x.S;
        d.nR = swap ? x.nS : x.nR;
        d.nS = swap ? x.nR : x.nS;
        d.orient = swap ? (kOrientSwap | g->rev_rpo) : 0u;
        d.voff = g->voff[x.graph];
        d.V = V;
        d.theta = x.theta;
        d.k = static_cast<uint32_t>(x.k);
        d.delta = x.delta == RN_DELTA_DEFAULT ? g->delta : x.delta;
        d.gdelta = g->gdelta[x.graph];
        d.wmin = g->w_min[x.graph];
        d.slack = ring_slack(g->wmean[x.graph]);
        d.sbits = static_cast<uint32_t>(sw);
        d.rbits = static_cast<uint32_t>(rw);
        d.hist = x.k ? nkcp * kHistWords : 0;
        nkcp += x.k ? 1 : 0;
        p.rbase[s] = static_cast<uint32_t>(rw);
        p.ebase[s + 1] = p.ebase[s] + static_cast<unsigned long long>(x.nS) + static_cast<unsigned long long>(x.nR);
        sw += round_up(words, 4);
        rw += words;
        if (sw >= 0xFFFFFFFFull || rw >= 0xFFFFFFFFull) return fail(RN_ERR_ARG, "too many vertices in one call");
        if (p.groups.empty() || p.groups.back().hb != hb[i] ||
            (hb[i] != kGlobalHB && p.groups.back().kcp != (x.k > 0)))
            p.groups.push_back(Group{hb[i], x.k > 0, true, s, s + 1, 0});
        Group &gr = p.groups.back();
        gr.kcp = gr.kcp || x.k > 0;
        gr.end = s + 1;
        gr.sources += static_cast<uint64_t>(d.nR);
        // compact tables: local ids below 2^24, and (theta-joins) every
        // distance within theta fits the compact word; a k-closest-pairs
        // search whose bound is larger moves on if it meets such a distance
        // (the compact 2^11 search's lists hold 64 entries: with buckets, delta
        // > 0, too few for its pending sets, so such groups keep wide tables)
        gr.compact = gr.compact && hb[i] >= kCompactMinHB && hb[i] <= kMaxHB && g->Vmax < kCompactVertices &&
                     (hb[i] != kCompactSmallRingHB || d.delta == 0) &&
                     g->A * (g->rev_rpo ? 2 : 1) < static_cast<int64_t>(kCompactArcs) &&
                     (x.k > 0 || x.theta <= compact_max_dist(hb[i]));
    }
    p.rbase[nq] = static_cast<uint32_t>(rw);
    p.total_elems = p.ebase[nq];
    p.sbits_words = static_cast<uint32_t>(sw);
    p.rbits_words = static_cast<uint32_t>(rw);
    for (const Group &gr : p.groups) {
        p.need_list0 |= gr.hb < kRetryHB1;
        p.need_list1 |= gr.hb < kMaxHB;
        p.any_global |= gr.hb == kGlobalHB;
    }
    // the bucket sort: theta-joins only, on graphs with varied weights, with
    // at most kMaxBins (query, dist) bins in all
    {
        uint64_t nb = 0;
        bool ok = !p.any_kcp;
        p.binbase.assign(static_cast<size_t>(nq) + 1, 0);
        for (int32_t i = 0; i < nq && ok; ++i) {
            p.binbase[i] = static_cast<uint32_t>(nb);
            nb += static_cast<uint64_t>(q[i].theta) + 1;
            ok = nb <= kMaxBins && g->varied[q[i].graph];
        }
        p.nbins = ok ? static_cast<uint32_t>(nb) : 0u;
        if (ok) p.binbase[nq] = p.nbins;
    }
    // the small sort: k-closest-pairs queries only, few candidates expected
    {
        bool all_kcp = nq > 0;
        uint64_t ksum = 0;
        for (int32_t i = 0; i < nq; ++i) {
            all_kcp = all_kcp && q[i].k > 0;
            ksum += static_cast<uint64_t>(std::max(q[i].k, 0));
        }
        p.small_sort = all_kcp && ksum <= kSmallSort / 2;
    }
    p.qb = nq > 1 ? bitlen(static_cast<uint64_t>(nq - 1)) : 0u;
    p.vb = std::max<uint32_t>(1u, bitlen(static_cast<uint64_t>(std::max(g->Vmax - 1, 0))));
    p.max_passes = std::max<uint32_t>(1u, (p.qb + std::max<uint32_t>(bitlen(dmax), 1u) + 2u * p.vb + 7u) / 8u);
    // call block: words, every region 64-word (256-byte) aligned
    p.off_qs = sizeof(CallCtl) / 4;
    p.off_sbits = round_up(p.off_qs + static_cast<size_t>(nq) * (sizeof(QueryState) / 4), 64);
    p.off_rbits = round_up(p.off_sbits + sw, 64);
    p.off_hists = round_up(p.off_rbits + rw, 64);
    p.off_work = round_up(p.off_hists + static_cast<size_t>(nkcp) * kHistWords, 64);   // one 256-byte line
    p.off_bins = p.off_work + 64;
    p.off_sort = round_up(p.off_bins + (p.nbins ? bucket_words(p.nbins) : 0), 64);
    p.block_words = p.off_sort + sort_hist_words();
    // the sort's histograms and digit totals are written whole before use;
    // the bucket sort needs its bin counts cleared (either way the clearing
    // covers the call state, histograms and the global tier's counter before
    // them)
    p.zero_words = p.nbins ? p.off_bins + p.nbins : p.off_bins;
    p.off_ebase = round_up(static_cast<size_t>(nq) * sizeof(QueryDesc), 16);
    p.off_rbase = round_up(p.off_ebase + static_cast<size_t>(nq + 1) * sizeof(unsigned long long), 16);
    p.off_perm = round_up(p.off_rbase + static_cast<size_t>(nq + 1) * sizeof(uint32_t), 16);
    p.off_binbase = round_up(p.off_perm + static_cast<size_t>(nq) * sizeof(uint32_t), 16);
    p.desc_bytes = p.off_binbase + (static_cast<size_t>(nq) + 1) * sizeof(uint32_t);
    return RN_OK;
}

rn_status ensure_gslots(Workspace &ws, int32_t Vmax, uint32_t want, hipStream_t s) {
    if (ws.d_gslots) return RN_OK;
    // one slot per concurrent global-tier search: as many as the call needs
    // (at least 64, so that a later call with more such searches still runs
    // them side by side), at most the workspace's cap and 48 GiB
    const size_t words = global_slot_words(Vmax);
    size_t n = std::max<size_t>(want, 64);
    n = std::min<size_t>(n, std::max<uint32_t>(ws.gslot_cap, 1));
    n = std::max<size_t>(1, std::min<size_t>(n, (size_t{48} << 30) / (4 * words)));
    RN_HIP(dev_alloc(&ws.d_gslots, n * words), "allocating global search slots");
    ws.n_gslots = static_cast<uint32_t>(n);
    RN_HIP(launch_fill_u32(ws.d_gslots, global_clear_words(ws.n_gslots, Vmax), 0xFFFFFFFFu, s),
           "clearing search slots");
    RN_HIP(hipStreamSynchronize(s), "clearing search slots");
    return RN_OK;
}

rn_status ensure_buffers(Workspace &ws, const Prepared &p) {
    if (ws.block_words < p.block_words) {
        dev_free(ws.d_block);
        ws.block_words = 0;
        const size_t words = p.block_words + p.block_words / 4;
        RN_HIP(dev_alloc(&ws.d_block, words), "allocating call buffers");
        ws.block_words = words;
    }
    if (ws.desc_bytes < p.desc_bytes) {
        dev_free(ws.d_desc);
        host_free(ws.h_desc);
        ws.desc_bytes = 0;
        const size_t bytes = std::max<size_t>(p.desc_bytes + p.desc_bytes / 4, 4096);
        RN_HIP(dev_alloc(&ws.d_desc, bytes), "allocating query descriptors");
        RN_HIP(hipHostMalloc(reinterpret_cast<void **>(&ws.h_desc), bytes, 0), "allocating query descriptors");
        ws.desc_bytes = bytes;
    }
    const size_t state_bytes = sizeof(CallCtl) + static_cast<size_t>(p.nq) * sizeof(QueryState);
    if (ws.h_state_bytes < state_bytes) {
        host_free(ws.h_state);
        ws.d_state_map = nullptr;
        ws.h_state_bytes = 0;
        const size_t bytes = std::max<size_t>(state_bytes + state_bytes / 4, 4096);
        RN_HIP(hipHostMalloc(reinterpret_cast<void **>(&ws.h_state), bytes, hipHostMallocMapped),
               "allocating the read-back buffer");
        ws.h_state_bytes = bytes;
        void *dp = nullptr;
        RN_HIP(hipHostGetDevicePointer(&dp, ws.h_state, 0), "mapping the read-back buffer");
        ws.d_state_map = static_cast<uint32_t *>(dp);
    }
    const size_t sw = stage_scratch_words(p.rbits_words);
    if (ws.stage_words < sw) {
        dev_free(ws.d_stage);
        ws.stage_words = 0;
        RN_HIP(dev_alloc(&ws.d_stage, sw + sw / 4), "allocating staging scratch");
        ws.stage_words = sw + sw / 4;
    }
    if (ws.src_cap < p.total_R) {
        dev_free(ws.d_src);
        dev_free(ws.d_srcq);
        for (int i = 0; i < kLists; ++i) {
            dev_free(ws.d_list[i]);
            dev_free(ws.d_listq[i]);
        }
        ws.src_cap = 0;
        const size_t cap = std::max<size_t>(p.total_R + p.total_R / 4, 1024);
        RN_HIP(dev_alloc(&ws.d_src, cap), "allocating the source list");
        RN_HIP(dev_alloc(&ws.d_srcq, cap), "allocating the source list");
        for (int i = 0; i < kLists; ++i) {
            RN_HIP(dev_alloc(&ws.d_list[i], cap), "allocating the re-run lists");
            RN_HIP(dev_alloc(&ws.d_listq[i], cap), "allocating the re-run lists");
        }
        ws.src_cap = cap;
    }
    if (ws.rec_cap == 0) {
        const unsigned long long cap = 1ull << 20;
        RN_HIP(dev_alloc(&ws.d_recs[0], cap), "allocating the record buffer");
        RN_HIP(dev_alloc(&ws.d_recs[1], cap), "allocating the record buffer");
        ws.rec_cap = cap;
    }
    if (!ws.fork) {
        RN_HIP(hipEventCreateWithFlags(&ws.fork, hipEventDisableTiming), "creating events");
        for (auto &e : ws.join) RN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "creating events");
        for (auto &e : ws.ev) RN_HIP(hipEventCreate(&e), "creating events");
    }
    return RN_OK;
}

rn_status grow_recs(Workspace &ws, unsigned long long need) {
    if (need >= kRecCapMax) return fail(RN_ERR_NOMEM, "a call may emit at most 2^31 - 1 records");
    const unsigned long long cap = std::min(kRecCapMax - 1, std::max(need + need / 4, 2 * ws.rec_cap));
    dev_free(ws.d_recs[0]);
    dev_free(ws.d_recs[1]);
    ws.rec_cap = 0;
    RN_HIP(dev_alloc(&ws.d_recs[0], cap), "growing the record buffer");
    RN_HIP(dev_alloc(&ws.d_recs[1], cap), "growing the record buffer");
    ws.rec_cap = cap;
    return RN_OK;
}

void fill_host_desc(const Prepared &p, uint8_t *h) {
    std::memcpy(h, p.qd.data(), static_cast<size_t>(p.nq) * sizeof(QueryDesc));
    std::memcpy(h + p.off_ebase, p.ebase.data(), p.ebase.size() * sizeof(unsigned long long));
    std::memcpy(h + p.off_rbase, p.rbase.data(), p.rbase.size() * sizeof(uint32_t));
    std::memcpy(h + p.off_perm, p.perm.data(), p.perm.size() * sizeof(uint32_t));
    std::memcpy(h + p.off_binbase, p.binbase.data(), p.binbase.size() * sizeof(uint32_t));
}

CallBuffers call_buffers(const Workspace &ws, const Prepared &p) {
    CallBuffers b;
    b.nq = p.nq;
    b.qd = reinterpret_cast<const QueryDesc *>(ws.d_desc);
    b.ebase = reinterpret_cast<const unsigned long long *>(ws.d_desc + p.off_ebase);
    b.rbase = reinterpret_cast<const uint32_t *>(ws.d_desc + p.off_rbase);
    b.perm = reinterpret_cast<const uint32_t *>(ws.d_desc + p.off_perm);
    b.binbase = reinterpret_cast<const uint32_t *>(ws.d_desc + p.off_binbase);
    b.nbins = p.nbins;
    b.bins = ws.d_block + p.off_bins;
    b.ctl = reinterpret_cast<CallCtl *>(ws.d_block);
    b.qs = reinterpret_cast<QueryState *>(ws.d_block + p.off_qs);
    b.sbits = ws.d_block + p.off_sbits;
    b.rbits = ws.d_block + p.off_rbits;
    b.rwords = p.rbits_words;
    b.hists = ws.d_block + p.off_hists;
    b.sort_hist = ws.d_block + p.off_sort;
    b.stage_scratch = ws.d_stage;
    b.src = ws.d_src;
    b.srcq = ws.d_srcq;
    for (int i = 0; i < kLists; ++i) {
        b.list[i] = ws.d_list[i];
        b.listq[i] = ws.d_listq[i];
    }
    b.recs[0] = ws.d_recs[0];
    b.recs[1] = ws.d_recs[1];
    b.rec_cap = ws.rec_cap;
    return b;
}

// ------------------------------------------------------------------ launch sequence
static void record(const rn_graph *g, Workspace &ws, bool timed, int which, hipStream_t s) {
    if (timed && g->profiling) (void)hipEventRecord(ws.ev[which], s);
}

static rn_status ensure_side_streams(Workspace &ws, size_t n) {
    for (size_t i = 0; i < n && i < static_cast<size_t>(kSide); ++i)
        if (!ws.side[i]) RN_HIP(hipStreamCreateWithFlags(&ws.side[i], hipStreamNonBlocking), "creating streams");
    return RN_OK;
}

// Enqueue the whole call on s (descriptors already on the device).  timed:
// record the profiling events (never during graph capture).
rn_status enqueue_call(rn_graph *g, Workspace &ws, const Prepared &p, rn_pair *out, int64_t cap, hipStream_t s,
                       bool timed, bool shared) {
    const CallBuffers b = call_buffers(ws, p);
    record(g, ws, timed, EV_START, s);
    RN_HIP(launch_fill_u32(ws.d_block, p.zero_words, 0u, s), "clearing call state");
    RN_HIP(launch_stage(b, p.total_elems, g->d_rank, s), "staging the queries");
    record(g, ws, timed, EV_STAGED, s);

    JoinArgs a;
    std::memset(&a, 0, sizeof(a));
    a.row_ptr = g->d_row_ptr;
    a.arcs = g->d_arcs;
    a.qd = b.qd;
    a.qs = b.qs;
    a.sbits = b.sbits;
    a.hists = b.hists;
    a.ctl = b.ctl;
    a.recs = b.recs[0];
    a.rec_cap = b.rec_cap;
    a.bins = p.nbins ? b.bins : nullptr;
    a.binbase = b.binbase;
    a.count_work = g->count_work ? 1 : 0;
    a.big_deg = g->big_deg ? 1 : 0;
    a.order = g->d_order;
    a.first = g->d_first;
    if (p.any_kcp) {
        JoinArgs k = a;
        k.src = b.src;
        k.srcq = b.srcq;
        k.sbeg = nullptr;
        k.send = &b.ctl->nsrc;
        RN_HIP(launch_kcp_seed(k, b, static_cast<uint32_t>(p.total_R), s), "seeding the k-closest-pairs bounds");
    }
    // first tiers, one launch per table size; several run side by side.  The
    // device gives a process few hardware queues (four), so the on-chip groups
    // share at most three streams (this one and two side streams, in turn),
    // and a group searched in the global tier from the start gets a side
    // stream of its own that the re-run tiers do not wait for: only the later
    // global launch, which takes the same slots, waits for it.
    const size_t ng = p.groups.size();
    if (ng > static_cast<size_t>(kSide) + 1) return fail(RN_ERR_DEVICE, "too many first-tier groups");
    const bool early_global = ng > 0 && p.groups[ng - 1].hb == kGlobalHB && ws.d_gslots != nullptr;
    const size_t non = ng - (early_global ? 1 : 0);                  // on-chip groups
    const size_t ons = shared ? 1 : std::max<size_t>(1, std::min<size_t>(non, 3));   // their streams
    const size_t gside = early_global && !shared ? 1 : 0;             // side stream 0: the global group
    const bool fork = ons > 1 || gside > 0;
    if (fork) {
        RN_TRY(ensure_side_streams(ws, gside + ons - 1));
        RN_HIP(hipEventRecord(ws.fork, s), "forking streams");
        for (size_t i = 0; i < gside + ons - 1; ++i) RN_HIP(hipStreamWaitEvent(ws.side[i], ws.fork, 0), "forking streams");
    }
    auto on_chip_stream = [&](size_t gi) { return gi % ons == 0 ? s : ws.side[gside + gi % ons - 1]; };
    for (size_t gi = 0; gi < ng; ++gi) {
        const Group &gr = p.groups[gi];
        JoinArgs t = a;
        t.src = b.src;
        t.srcq = b.srcq;
        t.sbeg = &b.qs[p.perm[gr.first]].src_start;
        t.send = gr.end < p.nq ? &b.qs[p.perm[gr.end]].src_start : &b.ctl->nsrc;
        if (early_global && gi == ng - 1) {
            // searches sure to outgrow every table: the global tier at once
            hipStream_t st = gside ? ws.side[0] : s;
            t.tier = 3;
            t.work = ws.d_block + p.off_work + 32;
            RN_HIP(launch_join_global(t, ws.d_gslots, ws.n_gslots, g->Vmax, static_cast<uint32_t>(gr.sources), st),
                   "launching the global relaxation");
        } else {
            // (without global-tier slots yet, a global group takes the largest
            // table, whose overflows get the slots and a re-run of the call)
            const int hbt = std::min(gr.hb, kMaxHB);
            const int li = retry_list_after(hbt);
            t.ovf = b.list[li];
            t.ovfq = b.listq[li];
            t.novf = &b.ctl->nlist[li];
            t.first_tier = 1;
            t.tier = 0;
            RN_HIP(launch_join(t, hbt, gr.kcp, gr.compact, static_cast<uint32_t>(gr.sources), !shared,
                               on_chip_stream(gi)),
                   "launching the relaxation");
        }
    }
    if (fork) {
        for (size_t i = 0; i < gside + ons - 1; ++i) RN_HIP(hipEventRecord(ws.join[i], ws.side[i]), "joining streams");
        for (size_t i = gside; i < gside + ons - 1; ++i) RN_HIP(hipStreamWaitEvent(s, ws.join[i], 0), "joining streams");
    }
    record(g, ws, timed, EV_TIER0, s);
    // re-runs: 2^11-slot tables, 2^14-slot tables, then the global tier
    const uint32_t maxs = static_cast<uint32_t>(p.total_R);
    for (int li = 0; li < 2; ++li) {
        if (li == 0 && !p.need_list0) continue;
        if (li == 1 && !p.need_list1) continue;
        JoinArgs t = a;
        t.src = b.list[li];
        t.srcq = b.listq[li];
        t.sbeg = nullptr;
        t.send = &b.ctl->nlist[li];
        t.ovf = b.list[li + 1];
        t.ovfq = b.listq[li + 1];
        t.novf = &b.ctl->nlist[li + 1];
        t.first_tier = 0;
        t.tier = 1 + li;
        // the re-run tiers take wide tables: they must hold any search the
        // first tiers sent on, whatever its distances (a compact 2^14 re-run
        // could only send those on to the global tier)
        RN_HIP(launch_join(t, li == 0 ? kRetryHB1 : kMaxHB, true, false, maxs, !shared, s),
               "launching the relaxation");
    }
    if (gside) RN_HIP(hipStreamWaitEvent(s, ws.join[0], 0), "joining streams");   // the early global launch
    if (ws.d_gslots) {   // (without slots the call is run again once they exist)
        JoinArgs t = a;
        t.src = b.list[2];
        t.srcq = b.listq[2];
        t.sbeg = nullptr;
        t.send = &b.ctl->nlist[2];
        t.tier = 3;
        t.work = ws.d_block + p.off_work;
        RN_HIP(launch_join_global(t, ws.d_gslots, ws.n_gslots, g->Vmax, maxs, s), "launching the global relaxation");
    }
    record(g, ws, timed, EV_RELAXED, s);
    if (p.any_kcp) RN_HIP(launch_select(b, s), "selecting candidates");
    const bool small = p.small_sort && p.nbins == 0;   // the small sort lays out the output itself
    if (!small) RN_HIP(launch_layout(b, p.any_kcp ? 1 : 0, p.qb, p.vb, p.nbins != 0, s), "laying out the output");
    record(g, ws, timed, EV_SELECTED, s);
    const size_t state_bytes = sizeof(CallCtl) + static_cast<size_t>(p.nq) * sizeof(QueryState);
    const uint32_t *state = reinterpret_cast<const uint32_t *>(ws.d_block);
    const uint32_t state_words = static_cast<uint32_t>(state_bytes / 4);
    bool published = false;   // the sort's kernel published the call state itself
    if (p.nbins) {
        RN_HIP(launch_bucket_sort(b, out, static_cast<unsigned long long>(cap), state, ws.d_state_map, state_words, s),
               "sorting pairs");
        published = true;
    } else if (small) {
        RN_HIP(launch_sort_small(b, p.qb, p.vb, out, static_cast<unsigned long long>(cap), state, ws.d_state_map,
                                 state_words, s),
               "sorting pairs");
        published = true;
    } else {
        RN_HIP(launch_sort_out(b, p.any_kcp ? 1 : 0, p.max_passes, p.vb, out, static_cast<unsigned long long>(cap), s),
               "sorting pairs");
    }
    record(g, ws, timed, EV_DONE, s);
    if (!published) RN_HIP(launch_publish(state, ws.d_state_map, state_words, s), "publishing the call state");
    return RN_OK;
}

rn_status enqueue_sort_fallback(const Workspace &ws, const Prepared &p, rn_pair *out, int64_t cap, hipStream_t s) {
    const CallBuffers b = call_buffers(ws, p);
    RN_HIP(launch_sort_out(b, 1, p.max_passes, p.vb, out, static_cast<unsigned long long>(cap), s), "sorting pairs");
    return RN_OK;
}

}  // namespace host
}  // namespace rn

namespace {


// The call's last kernel wrote its state into the mapped read-back buffer.
rn_status read_back(Workspace &ws, const Prepared &p, hipStream_t s) {
    (void)ws;
    (void)p;
    RN_HIP(hipStreamSynchronize(s), "waiting for the call");
    return RN_OK;
}

float elapsed(const rn_graph *g, const Workspace &ws, int a, int b) {
    float ms = 0.f;
    if (!g->profiling) return 0.f;
    if (hipEventElapsedTime(&ms, ws.ev[a], ws.ev[b]) != hipSuccess) return 0.f;
    return ms;
}

// Turn the read-back state into offsets / status / the return code (after
// the radix sort of a bucket-sorted call that found an oversized bin).
// Sets *regrow when the call must run again (records outgrew the buffer, or
// a search needed global-tier slots that did not exist yet).
rn_status finish(rn_graph *g, Workspace &ws, const Prepared &p, rn_pair *out, int64_t cap, int64_t *offsets,
                 int32_t *status, bool timed, bool *regrow, hipStream_t s) {
    const CallCtl &c = *reinterpret_cast<const CallCtl *>(ws.h_state);
    const QueryState *qs = reinterpret_cast<const QueryState *>(ws.h_state + sizeof(CallCtl));
    *regrow = false;
    if (c.nlist[2] > 0 && !ws.d_gslots) {
        // some search needed the global tier, which had no slots yet
        *regrow = true;
        RN_TRY(ensure_gslots(ws, g->Vmax, c.nlist[2], s));
    }
    if (c.npairs > ws.rec_cap && !*regrow) {
        *regrow = true;
        RN_TRY(grow_recs(ws, c.npairs));
    }
    if (*regrow) return RN_OK;
    if (c.resort) {
        RN_TRY(enqueue_sort_fallback(ws, p, out, cap, s));
        RN_HIP(hipStreamSynchronize(s), "waiting for the sort");
    }
    if (timed) {
        rn_stats &st = g->stats;
        st = rn_stats{};
        st.stage_ms = elapsed(g, ws, EV_START, EV_STAGED);
        st.relax_ms = elapsed(g, ws, EV_STAGED, EV_TIER0);
        st.retry_ms = elapsed(g, ws, EV_TIER0, EV_RELAXED);
        st.select_ms = elapsed(g, ws, EV_RELAXED, EV_SELECTED);
        st.sort_ms = elapsed(g, ws, EV_SELECTED, EV_DONE);
        st.total_ms = elapsed(g, ws, EV_START, EV_DONE);
        st.pairs = static_cast<int64_t>(c.npairs);
        st.arcs = static_cast<int64_t>(c.arcs);
        st.settled = static_cast<int64_t>(c.settled);
        st.retried = static_cast<int32_t>(c.nretry);
        st.global_searches = static_cast<int32_t>(c.nlist[2]);
        st.relax_launches = static_cast<int32_t>(p.groups.size()) + (p.need_list0 ? 1 : 0) + (p.need_list1 ? 1 : 0) + 1;
    }
    int bad = -1;
    uint32_t bad_err = 0;
    for (int32_t i = 0; i < p.nq; ++i) {
        if (qs[i].err && bad < 0) {
            bad_err = qs[i].err;
            if (p.qd[i].orient & kOrientSwap)   // duplicates were found in the swapped sets
                bad_err = (bad_err & ~(kErrDupR | kErrDupS)) | ((bad_err & kErrDupR) ? kErrDupS : 0u) |
                          ((bad_err & kErrDupS) ? kErrDupR : 0u);
        }
        if (offsets) offsets[i] = static_cast<int64_t>(qs[i].off);
        if (status) status[i] = qs[i].err ? RN_ERR_ARG : RN_OK;
        if (qs[i].err && bad < 0) bad = i;
    }
    if (offsets) offsets[p.nq] = static_cast<int64_t>(c.nout);
    if (c.nout > static_cast<unsigned long long>(cap)) return fail(RN_ERR_CAPACITY, "output buffer too small");
    if (bad >= 0)
        return fail(RN_ERR_ARG, (p.nq > 1 ? "query " + std::to_string(bad) + ": " : std::string()) +
                                    "invalid node sets:" + describe_err(bad_err));
    return RN_OK;
}

// One eager call on workspace ws (prepared p); retries when the record buffer
// was too small.
rn_status run_eager(rn_graph *g, Workspace &ws, const Prepared &p, rn_pair *out, int64_t cap, int64_t *offsets,
                    int32_t *status, hipStream_t s, bool timed) {
    RN_TRY(ensure_buffers(ws, p));
    for (int attempt = 0; attempt < 4; ++attempt) {
        fill_host_desc(p, ws.h_desc);
        RN_HIP(hipMemcpyAsync(ws.d_desc, ws.h_desc, p.desc_bytes, hipMemcpyHostToDevice, s), "uploading queries");
        RN_TRY(enqueue_call(g, ws, p, out, cap, s, timed));
        RN_TRY(read_back(ws, p, s));
        bool regrow = false;
        const rn_status st = finish(g, ws, p, out, cap, offsets, status, timed, &regrow, s);
        if (!regrow) return st;
    }
    return fail(RN_ERR_NOMEM, "record buffer did not settle");
}

rn_status run_batch(rn_graph *g, const rn_query *q, int32_t nq, rn_pair *out, int64_t cap, int64_t *offsets,
                    int32_t *status, hipStream_t s) {
    if (cap < 0 || (cap > 0 && !out)) return fail(RN_ERR_ARG, "bad output buffer");
    RN_TRY(check_queries(g, q, nq, status));
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    Prepared p;
    RN_TRY(prepare(g, q, nq, p));
    return run_eager(g, g->ws, p, out, cap, offsets, status, s, true);
}

rn_status run_single(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, uint32_t theta,
                     int32_t k, rn_pair *out, int64_t cap, int64_t *n_out, void *stream) {
    if (!n_out) return fail(RN_ERR_ARG, "n_out is NULL");
    *n_out = 0;
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    rn_query q;
    std::memset(&q, 0, sizeof(q));
    q.R = R;
    q.S = S;
    q.nR = nR;
    q.nS = nS;
    q.graph = 0;
    q.k = k;
    q.theta = theta;
    q.delta = RN_DELTA_DEFAULT;
    q.hash_log2 = 0;
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    int64_t off[2] = {0, 0};
    const rn_status st = run_batch(g, &q, 1, out, cap, off, nullptr, reinterpret_cast<hipStream_t>(stream));
    if (st == RN_OK || st == RN_ERR_CAPACITY) *n_out = off[1];
    return st;
}

rn_status validate_csr(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col, const uint32_t *w) {
    if (V < 1 || V >= 0x7FFFFFFF) return fail(RN_ERR_ARG, "V must be in [1, 2^31 - 2]");
    if (A < 0 || A >= 0x7FFFFFFFLL) return fail(RN_ERR_ARG, "A must be in [0, 2^31 - 1]");
    if (!row_ptr || (A > 0 && (!col || !w))) return fail(RN_ERR_ARG, "CSR array is NULL");
    if (row_ptr[0] != 0 || static_cast<int64_t>(row_ptr[V]) != A)
        return fail(RN_ERR_ARG, "row_ptr must start at 0 and end at A");
    for (int32_t x = 0; x < V; ++x)
        if (row_ptr[x + 1] < row_ptr[x]) return fail(RN_ERR_ARG, "row_ptr must be non-decreasing");
    for (int64_t a = 0; a < A; ++a)
        if (col[a] < 0 || col[a] >= V) return fail(RN_ERR_ARG, "col entry outside [0, V)");
    return RN_OK;
}

}  // namespace

extern "C" {

const char *rn_last_error(void) { return last_error().c_str(); }

const char *rn_version(void) { return "rn 0.2 (gfx950)"; }

}  // extern "C"

namespace {

// Graph index of global vertex x.
int32_t graph_of(const rn_graph *g, int32_t x) {
    return static_cast<int32_t>(std::upper_bound(g->voff.begin(), g->voff.end(), x) - g->voff.begin()) - 1;
}

// Build the device copy of the resident graphs from the host CSR (caller
// numbering), with global vertex x renumbered perm[x] (perm null: as is), and
// copy it into g->d_row_ptr / g->d_arcs (allocated on the first call; the
// size never changes, so plans captured earlier keep valid pointers).  Arc
// records carry their target's arc range; with g->rev_rpo the reversed arcs
// follow the forward ones.
rn_status upload_csr(rn_graph *g, const int32_t *perm) {
    const int32_t V = g->V;
    const int64_t A = g->A;
    const bool rev = g->rev_rpo != 0;
    std::vector<int32_t> rp, cl, rrp, rcl;
    std::vector<uint32_t> ww, rww;
    std::vector<ArcRec> arcs;
    try {
        rp.assign(static_cast<size_t>(V) + 1, 0);
        cl.resize(static_cast<size_t>(A));
        ww.resize(static_cast<size_t>(A));
        std::vector<int32_t> inv(static_cast<size_t>(V));
        for (int32_t x = 0; x < V; ++x) inv[perm ? perm[x] : x] = x;
        for (int32_t i = 0; i < V; ++i) rp[i + 1] = rp[i] + (g->row_ptr[inv[i] + 1] - g->row_ptr[inv[i]]);
        for (int32_t i = 0; i < V; ++i) {
            int32_t o = rp[i];
            for (int32_t a = g->row_ptr[inv[i]]; a < g->row_ptr[inv[i] + 1]; ++a, ++o) {
                cl[o] = perm ? perm[g->col[a]] : g->col[a];
                ww[o] = g->w[a];
            }
        }
        if (rev) {
            rrp.assign(static_cast<size_t>(V) + 1, 0);
            rcl.resize(static_cast<size_t>(A));
            rww.resize(static_cast<size_t>(A));
            for (int64_t a = 0; a < A; ++a) rrp[cl[a] + 1] += 1;
            for (int32_t x = 0; x < V; ++x) rrp[x + 1] += rrp[x];
            std::vector<int32_t> fill(rrp.begin(), rrp.end() - 1);
            for (int32_t x = 0; x < V; ++x)
                for (int32_t a = rp[x]; a < rp[x + 1]; ++a) {
                    const int32_t b = fill[cl[a]]++;
                    rcl[b] = x;
                    rww[b] = ww[a];
                }
        }
        arcs.resize(static_cast<size_t>(A) * (rev ? 2 : 1));
        for (int64_t a = 0; a < A; ++a) {
            const int32_t y = cl[a];
            arcs[a] = ArcRec{y, ww[a], rp[y], rp[y + 1]};
        }
        if (rev) {
            for (int64_t b = 0; b < A; ++b) {
                const int32_t y = rcl[b];
                arcs[A + b] = ArcRec{y, rww[b], static_cast<int32_t>(A) + rrp[y], static_cast<int32_t>(A) + rrp[y + 1]};
            }
            for (int32_t x = 0; x <= V; ++x) rp.push_back(static_cast<int32_t>(A) + rrp[x]);
        }
    } catch (...) {
        return fail(RN_ERR_NOMEM, "building the device graph");
    }
    // bit a: arc record a is the first lightest among the arcs from its tail
    // to its target (k-closest pairs count a pair of parallel arcs once)
    std::vector<uint32_t> first;
    try {
        first.assign((arcs.size() + 31) / 32, 0u);
        std::vector<int64_t> idx;
        const size_t nv = rp.size() - 1;   // forward rows, then the reversed ones
        for (size_t x = 0; x < nv; ++x) {
            const int64_t b = rp[x], e = rp[x + 1];
            if (e <= b) continue;
            if (e - b == 1) {
                first[static_cast<size_t>(b) >> 5] |= 1u << (b & 31);
                continue;
            }
            idx.resize(static_cast<size_t>(e - b));
            for (int64_t a = b; a < e; ++a) idx[static_cast<size_t>(a - b)] = a;
            std::sort(idx.begin(), idx.end(), [&](int64_t p, int64_t q) {
                const ArcRec &rp_ = arcs[static_cast<size_t>(p)], &rq = arcs[static_cast<size_t>(q)];
                if (rp_.y != rq.y) return rp_.y < rq.y;
                if (rp_.w != rq.w) return rp_.w < rq.w;
                return p < q;
            });
            for (size_t i = 0; i < idx.size(); ++i)
                if (i == 0 || arcs[static_cast<size_t>(idx[i])].y != arcs[static_cast<size_t>(idx[i - 1])].y)
                    first[static_cast<size_t>(idx[i]) >> 5] |= 1u << (idx[i] & 31);
        }
    } catch (...) {
        return fail(RN_ERR_NOMEM, "building the device graph");
    }
    hipError_t e = hipSuccess;
    if (!g->d_first && (e = dev_alloc(&g->d_first, std::max<size_t>(first.size(), 1))) != hipSuccess)
        return hip_fail(e, "uploading the graph");
    if (!first.empty() &&
        (e = hipMemcpy(g->d_first, first.data(), first.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "uploading the graph");
    if (!g->d_row_ptr && (e = dev_alloc(&g->d_row_ptr, rp.size())) != hipSuccess)
        return hip_fail(e, "uploading the graph");
    if (!g->d_arcs && (e = dev_alloc(&g->d_arcs, arcs.size())) != hipSuccess) return hip_fail(e, "uploading the graph");
    if ((e = hipMemcpy(g->d_row_ptr, rp.data(), rp.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
        (!arcs.empty() &&
         (e = hipMemcpy(g->d_arcs, arcs.data(), arcs.size() * sizeof(ArcRec), hipMemcpyHostToDevice)) != hipSuccess))
        return hip_fail(e, "uploading the graph");
    return RN_OK;
}

}  // namespace

extern "C" {

rn_status rn_graph_load_many(int32_t n, const int32_t *V, const int64_t *A, const int32_t *const *row_ptr,
                             const int32_t *const *col, const uint32_t *const *w, rn_graph **out) {
    if (!out) return fail(RN_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !V || !A || !row_ptr || !col || !w) return fail(RN_ERR_ARG, "need n >= 1 graphs and their arrays");
    int64_t totV = 0, totA = 0;
    for (int32_t i = 0; i < n; ++i) {
        const rn_status st = validate_csr(V[i], A[i], row_ptr[i], col[i], w[i]);
        if (st != RN_OK) return fail(st, "graph " + std::to_string(i) + ": " + t_err);
        totV += V[i];
        totA += A[i];
    }
    if (totV >= 0x7FFFFFFF) return fail(RN_ERR_ARG, "the graphs together exceed 2^31 - 2 vertices");
    if (totA >= 0x7FFFFFFFLL) return fail(RN_ERR_ARG, "the graphs together exceed 2^31 - 1 arcs");

    rn_graph *g = new (std::nothrow) rn_graph();
    if (!g) return fail(RN_ERR_NOMEM, "allocating the handle");
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "no HIP device");
    }
    g->ngraphs = n;
    g->V = static_cast<int32_t>(totV);
    g->A = totA;
    try {
        g->voff.assign(n + 1, 0);
        g->aoff.assign(n + 1, 0);
        g->w_min.assign(n, 0);
        g->gdelta.assign(n, 1);
        g->wmean.assign(n, 1.0);
        g->varied.assign(n, 0);
        g->row_ptr.resize(static_cast<size_t>(totV) + 1);
        g->col.resize(static_cast<size_t>(totA));
        g->w.resize(static_cast<size_t>(totA));
    } catch (...) {
        delete g;
        return fail(RN_ERR_NOMEM, "copying the CSR");
    }
    for (int32_t i = 0; i < n; ++i) {
        const int32_t vo = g->voff[i];
        const int64_t ao = g->aoff[i];
        g->voff[i + 1] = vo + V[i];
        g->aoff[i + 1] = ao + A[i];
        g->Vmax = std::max(g->Vmax, V[i]);
        for (int32_t x = 0; x < V[i]; ++x) g->row_ptr[vo + x] = static_cast<int32_t>(ao + row_ptr[i][x]);
        uint32_t wm = A[i] ? 0xFFFFFFFFu : 0u;
        for (int64_t a = 0; a < A[i]; ++a) {
            g->col[ao + a] = vo + col[i][a];
            g->w[ao + a] = w[i][a];
            wm = std::min(wm, w[i][a]);
        }
        g->w_min[i] = wm;
        // the global tier's buckets: 8 mean arc weights keep relaxations near
        // one per arc on road graphs at a few thousand rounds for a whole graph
        double wsum = 0;
        for (int64_t a = 0; a < A[i]; ++a) wsum += w[i][a];
        g->wmean[i] = A[i] ? std::max(1.0, wsum / static_cast<double>(A[i])) : 1.0;
        {
            std::vector<uint32_t> seen;
            for (int64_t a = 0; a < A[i] && seen.size() < 16; ++a)
                if (std::find(seen.begin(), seen.end(), w[i][a]) == seen.end()) seen.push_back(w[i][a]);
            g->varied[i] = seen.size() >= 16 ? 1 : 0;
        }
        const double gd = 8.0 * g->wmean[i];
        g->gdelta[i] = static_cast<uint32_t>(std::min(std::max(gd, 1.0), 2147483648.0));
    }
    g->row_ptr[totV] = static_cast<int32_t>(totA);
    // the reversed arcs (transpose), used when a query's S is smaller than its
    // R: the searches then run from S.  Symmetric graphs are their own
    // transpose and keep one copy.
    std::vector<int32_t> rrow(static_cast<size_t>(totV) + 1, 0), rcol;
    std::vector<uint32_t> rw;
    bool symmetric = true;
    try {
        rcol.resize(static_cast<size_t>(totA));
        rw.resize(static_cast<size_t>(totA));
    } catch (...) {
        delete g;
        return fail(RN_ERR_NOMEM, "transposing the CSR");
    }
    for (int64_t a = 0; a < totA; ++a) rrow[g->col[a] + 1] += 1;
    for (int32_t x = 0; x < totV; ++x) rrow[x + 1] += rrow[x];
    {
        std::vector<int32_t> fill(rrow.begin(), rrow.end() - 1);
        for (int32_t x = 0; x < totV; ++x)
            for (int32_t a = g->row_ptr[x]; a < g->row_ptr[x + 1]; ++a) {
                const int32_t b = fill[g->col[a]]++;
                rcol[b] = x;
                rw[b] = g->w[a];
            }
    }
    symmetric = rrow == g->row_ptr && rcol == g->col && rw == g->w;
    for (int32_t x = 0; x < totV && !g->big_deg; ++x)
        g->big_deg = g->row_ptr[x + 1] - g->row_ptr[x] > 0xFFFF || rrow[x + 1] - rrow[x] > 0xFFFF;
    const bool keep_rev = !symmetric && 2 * totA < 0x7FFFFFFFLL;
    g->can_swap = symmetric || keep_rev;
    g->rev_rpo = keep_rev ? static_cast<uint32_t>(totV + 1) : 0u;
    rcol.clear();
    rw.clear();
    // the resident copy, in the caller's numbering until rn_partition, and the
    // identity maps between the two numberings
    rn_status st = upload_csr(g, nullptr);
    if (st == RN_OK) {
        std::vector<int32_t> ident(static_cast<size_t>(totV));
        for (int32_t i = 0; i < totV; ++i) ident[i] = i - g->voff[graph_of(g, i)];
        std::vector<int32_t> rank_ident(ident);
        if ((e = dev_alloc(&g->d_rank, static_cast<size_t>(totV))) != hipSuccess ||
            (e = dev_alloc(&g->d_order, static_cast<size_t>(totV))) != hipSuccess ||
            (totV > 0 && ((e = hipMemcpy(g->d_rank, rank_ident.data(), ident.size() * sizeof(int32_t),
                                         hipMemcpyHostToDevice)) != hipSuccess ||
                          (e = hipMemcpy(g->d_order, ident.data(), ident.size() * sizeof(int32_t),
                                         hipMemcpyHostToDevice)) != hipSuccess)))
            st = hip_fail(e, "uploading the vertex maps");
    }
    if (st != RN_OK) {
        rn_graph_free(g);
        return st;
    }
    g->delta = 0;
    g->hash_log2 = 11;
    *out = g;
    return RN_OK;
}

rn_status rn_graph_load(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                        rn_graph **out) {
    return rn_graph_load_many(1, &V, &A, &row_ptr, &col, &w, out);
}

rn_status rn_objects_graph(const rn_graph *g, int32_t graph, const int32_t *arc, const uint32_t *offset, int32_t n,
                           rn_graph **out) {
    if (!out) return fail(RN_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (graph < 0 || graph >= g->ngraphs) return fail(RN_ERR_ARG, "graph index out of range");
    if (n < 0 || (n > 0 && (!arc || !offset))) return fail(RN_ERR_ARG, "need n >= 0 objects and their arrays");
    const int32_t vo = g->voff[graph], V = g->voff[graph + 1] - vo;
    const int64_t ao = g->aoff[graph], A = g->aoff[graph + 1] - ao;
    if (static_cast<int64_t>(V) + n >= 0x7FFFFFFF) return fail(RN_ERR_ARG, "too many objects");
    if (A + 2 * static_cast<int64_t>(n) >= 0x7FFFFFFFLL) return fail(RN_ERR_ARG, "too many objects");
    // the graph's own CSR (local ids)
    auto rp = [&](int32_t x) { return static_cast<int64_t>(g->row_ptr[vo + x]) - ao; };
    auto cl = [&](int64_t a) { return g->col[ao + a] - vo; };
    auto wt = [&](int64_t a) { return g->w[ao + a]; };
    // where each object sits: the arc naming its edge (of a road and its
    // two-way twin, the one with the smaller index; of parallel arcs with
    // equal ends and weight, the first), and its distance from that arc's tail
    struct Place {
        int64_t f, twin;
        uint32_t s;
    };
    std::vector<Place> pl;
    std::vector<std::vector<std::pair<uint32_t, int32_t>>> on_edge;   // per edge: (s, object)
    std::vector<int64_t> edge_of_arc;   // arc -> edge slot (-1: no object), for f and its twin
    try {
        pl.resize(static_cast<size_t>(n));
        edge_of_arc.assign(static_cast<size_t>(A), -1);
        for (int32_t i = 0; i < n; ++i) {
            const int64_t e = arc[i];
            if (e < 0 || e >= A) return fail(RN_ERR_ARG, "object " + std::to_string(i) + ": arc out of range");
            if (offset[i] > wt(e)) return fail(RN_ERR_ARG, "object " + std::to_string(i) + ": offset beyond its arc");
            const int32_t a = static_cast<int32_t>(std::upper_bound(g->row_ptr.begin() + vo, g->row_ptr.begin() + vo + V + 1,
                                                                    static_cast<int32_t>(ao + e)) -
                                                   (g->row_ptr.begin() + vo)) - 1;
            const int32_t b = cl(e);
            const uint32_t w = wt(e);
            int64_t ec = e, tw = -1;
            for (int64_t x = rp(a); x < rp(a + 1); ++x)
                if (cl(x) == b && wt(x) == w) { ec = x; break; }
            for (int64_t x = rp(b); x < rp(b + 1); ++x)
                if (cl(x) == a && wt(x) == w && x != ec) { tw = x; break; }
            Place &p = pl[static_cast<size_t>(i)];
            if (tw >= 0 && tw < ec) p = Place{tw, ec, w - offset[i]};
            else p = Place{ec, tw, offset[i]};
            if (edge_of_arc[static_cast<size_t>(p.f)] < 0) {
                edge_of_arc[static_cast<size_t>(p.f)] = static_cast<int64_t>(on_edge.size());
                if (p.twin >= 0) edge_of_arc[static_cast<size_t>(p.twin)] = static_cast<int64_t>(on_edge.size());
                on_edge.emplace_back();
            }
            on_edge[static_cast<size_t>(edge_of_arc[static_cast<size_t>(p.f)])].emplace_back(p.s, i);
        }
    } catch (...) {
        return fail(RN_ERR_NOMEM, "placing the objects");
    }
    for (auto &lst : on_edge) std::sort(lst.begin(), lst.end());
    // the subdivided graph: object i is vertex V + i; an edge's arc (and its
    // twin) is replaced by a chain through its objects in order of position
    const int32_t Vn = V + n;
    std::vector<int32_t> nrp, ncol;
    std::vector<uint32_t> nw;
    try {
        nrp.assign(static_cast<size_t>(Vn) + 1, 0);
        ncol.reserve(static_cast<size_t>(A + 2 * static_cast<int64_t>(n)));
        nw.reserve(static_cast<size_t>(A + 2 * static_cast<int64_t>(n)));
        for (int32_t x = 0; x < V; ++x) {
            for (int64_t e = rp(x); e < rp(x + 1); ++e) {
                const int64_t k = edge_of_arc[static_cast<size_t>(e)];
                if (k < 0) {
                    ncol.push_back(cl(e));
                    nw.push_back(wt(e));
                    continue;
                }
                const auto &lst = on_edge[static_cast<size_t>(k)];
                const Place &p0 = pl[static_cast<size_t>(lst.front().second)];
                if (e == p0.f) {           // tail -> first object
                    ncol.push_back(V + lst.front().second);
                    nw.push_back(lst.front().first);
                } else {                   // the twin: head -> last object
                    ncol.push_back(V + lst.back().second);
                    nw.push_back(wt(e) - lst.back().first);
                }
            }
            nrp[static_cast<size_t>(x) + 1] = static_cast<int32_t>(ncol.size());
        }
        // object rows: forward along the edge, then (two-way) back
        std::vector<std::pair<int64_t, size_t>> where(static_cast<size_t>(n));   // (edge, rank)
        for (size_t k = 0; k < on_edge.size(); ++k)
            for (size_t r = 0; r < on_edge[k].size(); ++r)
                where[static_cast<size_t>(on_edge[k][r].second)] = {static_cast<int64_t>(k), r};
        for (int32_t i = 0; i < n; ++i) {
            const Place &p = pl[static_cast<size_t>(i)];
            const auto &lst = on_edge[static_cast<size_t>(where[static_cast<size_t>(i)].first)];
            const size_t r = where[static_cast<size_t>(i)].second;
            const uint32_t w = wt(p.f);
            const int32_t tail = static_cast<int32_t>(std::upper_bound(g->row_ptr.begin() + vo,
                                                                      g->row_ptr.begin() + vo + V + 1,
                                                                      static_cast<int32_t>(ao + p.f)) -
                                                     (g->row_ptr.begin() + vo)) - 1;
            const int32_t head = cl(p.f);
            if (r + 1 < lst.size()) {
                ncol.push_back(V + lst[r + 1].second);
                nw.push_back(lst[r + 1].first - p.s);
            } else {
                ncol.push_back(head);
                nw.push_back(w - p.s);
            }
            if (p.twin >= 0) {
                if (r > 0) {
                    ncol.push_back(V + lst[r - 1].second);
                    nw.push_back(p.s - lst[r - 1].first);
                } else {
                    ncol.push_back(tail);
                    nw.push_back(p.s);
                }
            }
            nrp[static_cast<size_t>(V) + i + 1] = static_cast<int32_t>(ncol.size());
        }
    } catch (...) {
        return fail(RN_ERR_NOMEM, "building the graph with the objects");
    }
    const int64_t An = static_cast<int64_t>(ncol.size());
    return rn_graph_load(Vn, An, nrp.data(), ncol.data(), nw.data(), out);
}

void rn_graph_free(rn_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    g->ws.release();
    dev_free(g->d_row_ptr);
    dev_free(g->d_arcs);
    dev_free(g->d_rank);
    dev_free(g->d_order);
    dev_free(g->d_first);
    delete g;
}

int32_t rn_graph_num_vertices(const rn_graph *g) { return g ? g->V : 0; }
int64_t rn_graph_num_arcs(const rn_graph *g) { return g ? g->A : 0; }
int32_t rn_graph_count(const rn_graph *g) { return g ? g->ngraphs : 0; }

rn_status rn_graph_size(const rn_graph *g, int32_t i, int32_t *V, int64_t *A) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (i < 0 || i >= g->ngraphs) return fail(RN_ERR_ARG, "graph index out of range");
    if (V) *V = g->voff[i + 1] - g->voff[i];
    if (A) *A = g->aoff[i + 1] - g->aoff[i];
    return RN_OK;
}

rn_status rn_partition_host(int32_t V, int64_t A, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                            float alpha, int32_t max_leaf, int32_t *part_out, int32_t *order_out) {
    RN_TRY(validate_csr(V, A, row_ptr, col, w));
    if (!(alpha >= 0.f && alpha <= 1.f)) return fail(RN_ERR_ARG, "alpha must be in [0, 1]");
    if (max_leaf < 1) return fail(RN_ERR_ARG, "max_leaf must be >= 1");
    std::vector<int32_t> part, order;
    std::string msg;
    if (!partition_graph(V, row_ptr, col, w, alpha, max_leaf, part, order, msg)) return fail(RN_ERR_NOMEM, msg);
    if (part_out) std::memcpy(part_out, part.data(), static_cast<size_t>(V) * sizeof(int32_t));
    if (order_out) std::memcpy(order_out, order.data(), static_cast<size_t>(V) * sizeof(int32_t));
    return RN_OK;
}

rn_status rn_partition(rn_graph *g, float alpha, int32_t max_leaf, int32_t *part_out) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (!(alpha >= 0.f && alpha <= 1.f)) return fail(RN_ERR_ARG, "alpha must be in [0, 1]");
    if (max_leaf < 1) return fail(RN_ERR_ARG, "max_leaf must be >= 1");
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    const int32_t n = g->ngraphs;
    std::vector<std::vector<int32_t>> parts(n), orders(n);
    std::vector<std::string> msgs(n);
    std::vector<char> ok(n, 0);
    // graphs are independent: partition them on several host threads
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        for (int32_t i = next++; i < n; i = next++) {
            const int32_t vo = g->voff[i], V = g->voff[i + 1] - vo;
            const int64_t ao = g->aoff[i], A = g->aoff[i + 1] - ao;
            std::vector<int32_t> rp(static_cast<size_t>(V) + 1), cl(static_cast<size_t>(A));
            for (int32_t x = 0; x <= V; ++x) rp[x] = static_cast<int32_t>(g->row_ptr[vo + x] - ao);
            for (int64_t a = 0; a < A; ++a) cl[a] = g->col[ao + a] - vo;
            ok[i] = partition_graph(V, rp.data(), cl.data(), g->w.data() + ao, alpha, max_leaf, parts[i], orders[i],
                                    msgs[i]) ? 1 : 0;
        }
    };
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const unsigned nt = std::min<unsigned>(hw, static_cast<unsigned>(n));
    std::vector<std::thread> pool;
    try {
        for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work);
    } catch (...) {
    }
    work();
    for (auto &t : pool) t.join();
    for (int32_t i = 0; i < n; ++i)
        if (!ok[i]) return fail(RN_ERR_NOMEM, msgs[i]);
    // within a leaf, keep the caller's order (the leaves are what the
    // partition contributes; a graph numbered with locality keeps it inside them)
    for (int32_t i = 0; i < n; ++i) {
        std::vector<int32_t> &o = orders[i];
        const std::vector<int32_t> &pt = parts[i];
        for (size_t b = 0; b < o.size();) {
            size_t e = b + 1;
            while (e < o.size() && pt[o[e]] == pt[o[b]]) ++e;
            std::sort(o.begin() + static_cast<std::ptrdiff_t>(b), o.begin() + static_cast<std::ptrdiff_t>(e));
            b = e;
        }
    }
    std::vector<int32_t> rank(static_cast<size_t>(g->V)), order(static_cast<size_t>(g->V));
    int32_t leaf0 = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t vo = g->voff[i], V = g->voff[i + 1] - vo;
        int32_t nleaf = 0;
        for (int32_t r = 0; r < V; ++r) {
            order[vo + r] = orders[i][r];
            rank[vo + orders[i][r]] = r;
        }
        for (int32_t x = 0; x < V; ++x) {
            nleaf = std::max(nleaf, parts[i][x] + 1);
            if (part_out) part_out[vo + x] = leaf0 + parts[i][x];
        }
        leaf0 += nleaf;
    }
    // the resident copy of a graph is renumbered in leaf order (in place: plans
    // captured earlier stay valid) where that keeps the two ends of its arcs
    // closer together than the loaded numbering does: mean |id(x) - id(y)|
    // over the arcs, which ranks the numberings of the synthetic road graphs
    // as their search times do (row by row 542, leaf order 1 499, shuffled
    // 349 000 on the 1024^2 graph); otherwise it stays as loaded
    std::vector<int32_t> perm(static_cast<size_t>(g->V));
    g->renumbered.assign(static_cast<size_t>(n), 0);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t vo = g->voff[i], V = g->voff[i + 1] - vo;
        double as_loaded = 0, leaf = 0;
        for (int32_t x = 0; x < V; ++x)
            for (int32_t a = g->row_ptr[vo + x]; a < g->row_ptr[vo + x + 1]; ++a) {
                const int32_t y = g->col[a] - vo;
                as_loaded += std::abs(static_cast<double>(x) - y);
                leaf += std::abs(static_cast<double>(rank[vo + x]) - rank[vo + y]);
            }
        g->renumbered[i] = leaf < as_loaded ? 1 : 0;
        for (int32_t x = 0; x < V; ++x) {
            if (!g->renumbered[i]) {
                rank[vo + x] = x;
                order[vo + x] = x;
            }
            perm[vo + x] = vo + rank[vo + x];
        }
    }
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    RN_HIP(hipDeviceSynchronize(), "waiting for the device");
    RN_TRY(upload_csr(g, perm.data()));
    RN_HIP(hipMemcpy(g->d_rank, rank.data(), rank.size() * sizeof(int32_t), hipMemcpyHostToDevice), "uploading ranks");
    RN_HIP(hipMemcpy(g->d_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice),
           "uploading ranks");
    return RN_OK;
}

int32_t rn_graph_renumbered(const rn_graph *g, int32_t graph) {
    if (!g || graph < 0 || graph >= g->ngraphs || g->renumbered.empty()) return 0;
    return g->renumbered[static_cast<size_t>(graph)];
}

rn_status rn_set_tuning(rn_graph *g, int64_t delta, int32_t hash_log2) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (delta > static_cast<int64_t>(kMaxDist)) return fail(RN_ERR_ARG, "delta out of range");
    if (hash_log2 >= 0 && !join_tier_supported(hash_log2)) return fail(RN_ERR_ARG, "hash_log2 must be in [8, 14]");
    if (delta >= 0) g->delta = static_cast<uint32_t>(delta);
    if (hash_log2 >= 0) {
        g->hash_log2 = hash_log2;
        g->hash_auto = false;
    }
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

rn_status rn_dist_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, uint32_t theta,
                       rn_pair *out, int64_t cap, int64_t *n_out, void *stream) {
    return run_single(g, R, nR, S, nS, theta, 0, out, cap, n_out, stream);
}

rn_status rn_kcp_join(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, int32_t k,
                      rn_pair *out, int64_t cap, int64_t *n_out, void *stream) {
    if (n_out) *n_out = 0;
    if (k < 1 || k > (1 << 24)) return fail(RN_ERR_ARG, "k must be in [1, 2^24]");
    return run_single(g, R, nR, S, nS, kMaxDist, k, out, cap, n_out, stream);
}

rn_status rn_join_batch(rn_graph *g, const rn_query *q, int32_t nq, rn_pair *out, int64_t cap, int64_t *offsets,
                        int32_t *status, void *stream) {
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (!offsets) return fail(RN_ERR_ARG, "offsets is NULL");
    if (nq >= 1 && nq <= kMaxQueries) std::fill(offsets, offsets + nq + 1, 0);
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    return run_batch(g, q, nq, out, cap, offsets, status, reinterpret_cast<hipStream_t>(stream));
}

rn_status rn_autotune(rn_graph *g, rn_query *q, int32_t nq, int32_t sample, void *stream) {
    if (sample < 1) return fail(RN_ERR_ARG, "sample must be >= 1");
    RN_TRY(check_queries(g, q, nq, nullptr));
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool prof = g->profiling, work = g->count_work;
    g->profiling = true;
    g->count_work = false;
    rn_status result = RN_OK;
    for (int32_t i = 0; i < nq && result == RN_OK; ++i) {
        rn_query t = q[i];
        t.nR = std::min(t.nR, sample);
        const uint32_t wm = std::max(1u, g->w_min[t.graph]);
        const uint32_t deltas[3] = {0u, wm, 4u * wm};
        const int hbs_join[4] = {9, 10, 11, 12};
        const int hbs_kcp[3] = {8, 9, 10};
        const int *hbs = t.k ? hbs_kcp : hbs_join;
        const int nh = t.k ? 3 : 4;
        float best = 3.4e38f;
        uint32_t best_delta = g->delta;
        int best_hb = t.k ? kMinHB : g->hash_log2;
        for (int di = 0; di < 4 && result == RN_OK; ++di) {
            for (int hi = 0; hi < (di < 3 ? nh : 1) && result == RN_OK; ++hi) {
                // the fourth setting: the global tier from the start (its
                // buckets have their own width, so delta does not apply)
                t.delta = di < 3 ? deltas[di] : g->delta;
                t.hash_log2 = di < 3 ? hbs[hi] : kGlobalHB;
                Prepared p;
                result = prepare(g, &t, 1, p);
                if (result != RN_OK) break;
                float ms = 3.4e38f;
                for (int rep = 0; rep < 3 && result == RN_OK; ++rep) {
                    result = run_eager(g, g->ws, p, nullptr, 0, nullptr, nullptr, s, true);
                    if (result == RN_ERR_CAPACITY) result = RN_OK;   // counts only: no output wanted
                    if (result == RN_ERR_ARG) {
                        result = RN_OK;   // invalid node sets: keep the defaults for this query
                        break;
                    }
                    if (rep > 0) ms = std::min(ms, g->stats.relax_ms + g->stats.retry_ms);
                }
                if (ms < best) {
                    best = ms;
                    best_delta = t.delta;
                    best_hb = t.hash_log2;
                }
            }
        }
        q[i].delta = best_delta;
        q[i].hash_log2 = best_hb;
    }
    g->profiling = prof;
    g->count_work = work;
    return result;
}

void rn_plan_free(rn_plan *p) {
    if (!p) return;
    if (p->g) (void)hipSetDevice(p->g->device);
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    p->ws.release();
    delete p;
}

}  // extern "C"

namespace {

// Capture the plan's call into a graph (descriptors already uploaded).
rn_status capture_plan(rn_plan *pl, const Prepared &p) {
    rn_graph *g = pl->g;
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec), pl->exec = nullptr;
    if (pl->graph) (void)hipGraphDestroy(pl->graph), pl->graph = nullptr;
    RN_HIP(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal), "starting the capture");
    const rn_status st = enqueue_call(g, pl->ws, p, pl->out, pl->cap, pl->cap_stream, false);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(pl->cap_stream, &graph);
    if (st != RN_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "ending the capture");
    pl->graph = graph;
    RN_HIP(hipGraphInstantiate(&pl->exec, graph, nullptr, nullptr, 0), "instantiating the graph");
    return RN_OK;
}

// Eager run to size the buffers, then capture.
rn_status plan_build(rn_plan *pl, const Prepared &p, hipStream_t s, int64_t *offsets, int32_t *status) {
    const rn_status st = run_eager(pl->g, pl->ws, p, pl->out, pl->cap, offsets, status, s, false);
    if (st != RN_OK && st != RN_ERR_CAPACITY && st != RN_ERR_ARG) return st;
    RN_TRY(capture_plan(pl, p));
    return st;
}

}  // namespace

extern "C" {

rn_status rn_plan_create(rn_graph *g, const rn_query *q, int32_t nq, rn_pair *out, int64_t cap, void *stream,
                         rn_plan **plan) {
    if (!plan) return fail(RN_ERR_ARG, "plan is NULL");
    *plan = nullptr;
    if (cap < 0 || (cap > 0 && !out)) return fail(RN_ERR_ARG, "bad output buffer");
    RN_TRY(check_queries(g, q, nq, nullptr));
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    rn_plan *pl = new (std::nothrow) rn_plan();
    if (!pl) return fail(RN_ERR_NOMEM, "allocating the plan");
    pl->g = g;
    pl->out = out;
    pl->cap = cap;
    pl->q.assign(q, q + nq);
    Prepared &p = pl->prep;
    rn_status st = prepare(g, q, nq, p);
    hipError_t e = hipSuccess;
    if (st == RN_OK && (e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        st = hip_fail(e, "creating the capture stream");
    if (st == RN_OK) {
        st = plan_build(pl, p, reinterpret_cast<hipStream_t>(stream), nullptr, nullptr);
        if (st == RN_ERR_CAPACITY || st == RN_ERR_ARG) st = RN_OK;   // reported again by every run
    }
    if (st != RN_OK) {
        const std::string msg = t_err;
        rn_plan_free(pl);
        return fail(st, msg);
    }
    *plan = pl;
    return RN_OK;
}

rn_status rn_plan_run(rn_plan *pl, int64_t *offsets, int32_t *status, void *stream) {
    if (!pl || !pl->exec) return fail(RN_ERR_ARG, "plan is NULL");
    if (!offsets) return fail(RN_ERR_ARG, "offsets is NULL");
    rn_graph *g = pl->g;
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Prepared &p = pl->prep;
    RN_HIP(hipGraphLaunch(pl->exec, s), "launching the graph");
    RN_TRY(read_back(pl->ws, p, s));
    bool regrow = false;
    const rn_status st = finish(g, pl->ws, p, pl->out, pl->cap, offsets, status, false, &regrow, s);
    if (!regrow) return st;
    // the records outgrew the buffer (grown by finish): run eagerly, re-capture
    return plan_build(pl, p, s, offsets, status);
}

}  // extern "C"
