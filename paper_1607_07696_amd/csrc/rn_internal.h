// rn_internal.h -- types shared by the library's host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rn.h"

namespace rn {

constexpr uint32_t kInf = 0xFFFFFFFFu;     // unreachable / empty distance
constexpr uint32_t kMaxDist = 0xFFFFFFFEu; // largest representable distance

// Argument errors found on the device while staging a query (QueryState::err bits).
enum : uint32_t {
    kErrRange = 1u,    // an id outside [0, V)
    kErrDupR = 2u,     // a duplicate in R
    kErrDupS = 4u,     // a duplicate in S
    kErrOverlap = 8u,  // a vertex in both R and S
};

// On-chip table sizes (log2 of the slot count) a search may start with, and
// the two fixed re-run sizes: a search that outgrows its first table is re-run
// with a 2^11-slot table when it started below that, else with 2^14 slots; one
// that outgrows 2^14 slots moves to the global-memory tier, which takes any
// search.  Re-run lists: 0 -> 2^11, 1 -> 2^14, 2 -> global.
constexpr int kMinHB = 8;
constexpr int kMaxHB = 14;
constexpr int kRetryHB1 = 11;
// First-tier "table size" of queries whose searches run in the global tier
// from the start (RN_TABLE_GLOBAL).
constexpr int kGlobalHB = kMaxHB + 1;
constexpr int kLists = 3;
inline int retry_list_after(int hb) { return hb < kRetryHB1 ? 0 : (hb < kMaxHB ? 1 : 2); }

// k-closest pairs: distances are counted in log-spaced bins (16 per octave:
// exact below 16, then 16 steps per power of two); the upper edge of the bin
// holding the k-th count bounds the k-th smallest distance from above.
constexpr uint32_t kDistBins = 512;   // 464 used

// Histogram region of one k-closest-pairs query (words): the weights of direct
// R-S arcs | the distances of emitted pairs | for each search tier, the first
// tentative distance of every (source, S member) pair its searches discovered |
// the four discovery counts.  Each histogram counts a pair at most once, and
// every value counted is the length of a real path, so each one alone bounds
// the k-th smallest distance from above once it holds k counts.
constexpr uint32_t kHistSeed = 0;
constexpr uint32_t kHistEmit = kDistBins;
constexpr uint32_t kHistProbe = 2 * kDistBins;      // + tier * kDistBins
constexpr uint32_t kHistCount = 6 * kDistBins;      // + tier
constexpr uint32_t kHistWords = 6 * kDistBins + 64;

// One query of a call as the kernels read it (uploaded per call).  Ids in R
// and S are local to the query's graph; the graph's vertices are the global
// ids voff .. voff + V - 1 of the resident CSR.
struct QueryDesc {
    const int32_t *R;           // device int32[nR]
    const int32_t *S;           // device int32[nS]
    int32_t nR, nS;
    int32_t voff, V;
    uint32_t theta;             // distance bound (inclusive)
    uint32_t k;                 // 0: theta-join; else the k closest pairs within theta
    uint32_t delta;             // bucket width (0 = one bucket)
    uint32_t sbits;             // word offset of the query's S bitmap in the S-bitmap pool
    uint32_t rbits;             // word offset of the query's rank bitmap in the rank-bitmap pool
    uint32_t hist;              // k > 0: word offset of its histogram region in the histogram pool
    uint32_t gdelta;            // bucket width of the global-memory tier (>= 1)
    uint32_t orient;            // bit 31: the caller's R and S are swapped here (the search runs
                                // from S over the reversed arcs); bits 0-30: row pointer offset
                                // of the arcs searched (0: the forward CSR)
    uint32_t wmin;              // lightest arc weight of the query's graph
    uint32_t slack;             // delta = 0: a step of the on-chip search puts back the vertices
                                // more than this above its least distance (kInf: none)
    uint32_t pad[2];
};
static_assert(sizeof(QueryDesc) == 80, "QueryDesc is 80 bytes");
constexpr uint32_t kOrientSwap = 1u << 31;

// Per-query device state of one call.  Zeroed first.
struct QueryState {
    uint32_t err;               // kErr* bits
    uint32_t bound;             // k > 0: current distance bound (seeded, then lowered)
    uint32_t src_start;         // first entry of the query's sources in the source list
    uint32_t direct;            // k > 0: 1 when every pair within the seeded bound is a direct arc
                                // (the bound is below twice the lightest arc): one thread per
                                // source answers the query, and its searches are skipped
    unsigned long long npairs;  // records the query emitted
    unsigned long long nsel;    // records kept by the final bound
    unsigned long long start;   // first kept record of the query in the sorted order
    unsigned long long nout;    // pairs written for the query
    unsigned long long off;     // first output position of the query
    unsigned long long pad2;
};
static_assert(sizeof(QueryState) == 64, "QueryState is 64 bytes");

// Control block of one call.  Zeroed first; QueryState[nq] follows it.
struct CallCtl {
    uint32_t err;               // OR of every query's error bits
    uint32_t nsrc;              // sources staged
    unsigned long long npairs;  // records emitted (may exceed the record buffer)
    uint32_t nlist[kLists];     // sources queued on each re-run list
    uint32_t nretry;            // sources that outgrew their first table
    unsigned long long arcs;    // work count: out-arcs of every settled (source, vertex)
    unsigned long long settled; // work count: settled (source, vertex) pairs
    unsigned long long nsel;    // records kept by the final bounds
    unsigned long long nout;    // pairs owed to the caller
    uint32_t sort_db;           // distance bits of the sort key
    uint32_t sort_passes;       // 8-bit digit passes the sort needs
    uint32_t nchunks;           // bucket sort: 64-record chunks over all bins
    uint32_t resort;            // the call's sort left the output to the radix sort (a bucket-sort bin
                                //   above kBucketRankMax records, or more than kSmallSort candidates)
};
static_assert(sizeof(CallCtl) == 80, "CallCtl is 80 bytes");

// One emitted (u, v, dist) of query q, ids local to the query's graph.
struct alignas(16) Rec {
    int32_t u;
    int32_t v;
    uint32_t d;
    uint32_t q;
};

// One arc as the relaxation kernels read it: target, weight, and the target's
// own arc range, so expanding a vertex needs no separate row_ptr lookup.
// Vertex ids and arc indices are global across the resident graphs.  A handle
// whose graphs are not symmetric also keeps the reversed arcs: row pointers
// [V+1, 2V+2) and arcs [A, 2A) after the forward ones.
struct alignas(16) ArcRec {
    int32_t y;
    uint32_t w;
    int32_t ybeg;
    int32_t yend;
};

// Arguments of one relaxation launch.  The launch searches from the sources
// src[b .. e) with b = *sbeg (0 if sbeg is null) and e = *send.
struct JoinArgs {
    const int32_t *row_ptr;     // resident CSR row pointers (global ids)
    const ArcRec *arcs;
    const QueryDesc *qd;
    QueryState *qs;
    const uint32_t *sbits;      // S-bitmap pool
    uint32_t *hists;            // histogram pool (k-closest pairs)
    const int32_t *src;         // sources (global ids) and their queries
    const uint32_t *srcq;
    const uint32_t *sbeg;
    const uint32_t *send;
    CallCtl *ctl;
    Rec *recs;                  // emitted records
    unsigned long long rec_cap;
    int32_t *ovf;               // where searches that outgrow this tier are queued
    uint32_t *ovfq;
    uint32_t *novf;
    uint32_t *bins;             // bucket sort: per-bin record counts, kept as records are stored (else null)
    const uint32_t *binbase;    //   first bin of each query
    int32_t first_tier;         // 1: count re-queued searches in ctl->nretry
    int32_t tier;               // 0 first table, 1 and 2 the re-run tables, 3 the global tier
    int32_t count_work;         // 1: accumulate ctl->arcs / ctl->settled
    int32_t big_deg;            // 1: some vertex has 2^16 or more arcs (searches reaching one move on)
    const int32_t *order;       // global vertex of the device copy -> local id in the caller's numbering
    const uint32_t *first;      // bit a: arc a is the first lightest of the arcs from its tail to its
                                //   target (parallel arcs give one pair, at that arc's weight)
    uint32_t *work;             // global tier: counter of sources claimed past the grid (zero at the start)
};

// State of the global-memory tier: n slots (one per concurrent block), V the
// largest graph's vertex count, laid out array by array across the slots:
// word[n][V] (64-bit: distance and queue round) | frontier spill[n][V] |
// second frontier spill[n][V] | touched[n][V] | far list[n][V] (32-bit).
// Between searches every word is all ones (the first array, filled with ones
// at allocation: global_clear_words words).
inline size_t global_slot_words(int32_t V) { return 6 * static_cast<size_t>(V); }
inline size_t global_clear_words(uint32_t nslots, int32_t V) { return 2 * static_cast<size_t>(nslots) * V; }

// Host-side description of the call buffers the launch sequence uses.
struct CallBuffers {
    int32_t nq;
    const QueryDesc *qd;        // [nq]
    const unsigned long long *ebase;   // [nq+1] prefix of nS + nR in staging order
    const uint32_t *rbase;      // [nq+1] rank-pool word prefix in staging order
    const uint32_t *perm;       // [nq] query at each staging position
    CallCtl *ctl;               // followed by QueryState[nq]
    QueryState *qs;
    uint32_t *sbits;            // S-bitmap pool
    uint32_t *rbits;            // rank-bitmap pool
    uint32_t rwords;            // its words
    uint32_t *hists;            // histogram pool
    uint32_t *sort_hist;        // sort_hist_words() words
    const uint32_t *binbase;    // bucket sort: [nq+1] first bin of each query (query order)
    uint32_t nbins;             //   bins (query, dist); 0 when the call uses the radix sort
    uint32_t *bins;             //   count[nbins] (zeroed) | start[nbins] | cursor[nbins] | chunk start[nbins+1]
    uint32_t *stage_scratch;    // stage_scratch_words(rwords) words
    int32_t *src;               // source list and its queries
    uint32_t *srcq;
    int32_t *list[kLists];      // re-run lists and their queries
    uint32_t *listq[kLists];
    Rec *recs[2];
    unsigned long long rec_cap;
};

// ---- launchers (rn_kernels.hip); all enqueue on stream s
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
// Copy a call's state (words 32-bit words from device memory) into mapped
// pinned host memory (dst: its device address), as the call's last kernel:
// the host then only waits for the stream, with no copy queued after the call.
hipError_t launch_publish(const uint32_t *src, uint32_t *dst, uint32_t words, hipStream_t s);

// Validate every query's R and S, set the S bitmaps and rank bitmaps (both in
// the device copy's numbering), and list the sources query by query (staging
// order) in that numbering.  rank: caller's global vertex -> local id in the
// device copy (nullptr: identity).  max_elems: sum of nS + nR over the queries.
hipError_t launch_stage(const CallBuffers &b, unsigned long long max_elems, const int32_t *rank, hipStream_t s);
size_t stage_scratch_words(size_t rwords);

// Relaxation at the on-chip tier with table size 2^hash_log2.  generic =
// false: every source belongs to a theta-join (the kernel variant without the
// k-closest-pairs code).  compact: the table packs each slot into one 32-bit
// word (every graph of the call has fewer than kCompactVertices vertices; a
// search reaching a distance above compact_max_dist(hash_log2), or a probe
// sequence longer than the word records, is queued for the next tier like
// one that outgrows its table).  persistent: a device-filling grid of blocks
// that loop over the sources; else one block per source.
constexpr int32_t kCompactVertices = 1 << 24;
// ... and the handle's arc records (forward and reversed) number fewer than
// kCompactArcs: a compact search's window map names an arc in 26 bits
constexpr uint32_t kCompactArcs = 1u << 26;
// bits of a compact word that hold a slot's probe distance (longer probe
// sequences send the search on), and the largest distance the word holds
constexpr uint32_t compact_disp_bits(int hash_log2) { return hash_log2 >= 14 ? 5u : 4u; }
constexpr uint32_t compact_max_dist(int hash_log2) {
    return (1u << (7u + static_cast<uint32_t>(hash_log2) - compact_disp_bits(hash_log2))) - 2u;
}
// Compact tables are used from this size on.  Their 12 KiB (2^11) and 8 KiB
// (2^10) per search hold 12 and 18 searches per CU against the wide tables' 8
// and 12, which outweighs their longer arithmetic (2^11 at theta = 3000:
// 0.224 against 0.268 ms); at 2^9 both hold 18 or more, and the wide table's
// simpler arithmetic is faster.
constexpr int kCompactMinHB = 10;
// The compact table size whose search takes a 128-entry ring (lists of 64).
constexpr int kCompactSmallRingHB = 11;
hipError_t launch_join(const JoinArgs &a, int hash_log2, bool generic, bool compact, uint32_t max_sources,
                       bool persistent, hipStream_t s);
int join_tier_supported(int hash_log2);
// The global-memory tier: one block per source, nslots slots of
// global_slot_words(Vmax) words in the layout above.
hipError_t launch_join_global(const JoinArgs &a, uint32_t *slots, uint32_t nslots, int32_t Vmax,
                              uint32_t max_sources, hipStream_t s);

// k closest pairs: seed every k-query's bound from the direct arcs between its
// R and S, capped by its theta; answer the queries whose seeded bound is below
// twice their lightest arc from the direct arcs alone (QueryState::direct).
hipError_t launch_kcp_seed(const JoinArgs &a, const CallBuffers &b, uint32_t max_sources, hipStream_t s);

// Keep the records within their query's final bound (into recs[1]).
hipError_t launch_select(const CallBuffers &b, hipStream_t s);

// Per-query segments of the sorted records and of the output, the key layout
// of the sort (ctl->sort_db, ctl->sort_passes); selected: records were
// filtered by launch_select (else every emitted record is kept in place).
// bins: the call takes the bucket sort, whose bin scan runs in the same block.
hipError_t launch_layout(const CallBuffers &b, int selected, uint32_t qb, uint32_t vb, bool bins, hipStream_t s);

// Sort the kept records by (query, dist, u, v) and write each query's first
// nout pairs to out at its offset, unless the records outgrew the buffer or
// the total exceeds user_cap.  Launches max_passes digit passes; those beyond
// ctl->sort_passes return at once.
hipError_t launch_sort_out(const CallBuffers &b, int selected, uint32_t max_passes, uint32_t vb,
                           rn_pair *out, unsigned long long user_cap, hipStream_t s);
size_t sort_hist_words();
constexpr uint32_t kSortPassesMax = 16;

// Queries per call.  Query numbers fit in 16 bits: the bucket sort keeps a
// record's place in its bin in the upper half of its 32-bit query field.
constexpr int32_t kMaxQueries = 65536;

// Bucket sort, for calls of theta-joins only whose bins (query, dist), theta+1
// per query, number at most kMaxBins: the relaxation kernels count the records
// per bin as they store them (the count's old value is the record's place in
// its bin); the layout launch scans the counts; the scatter copies each record
// to its place, then order each bin by (u, v) by counting the smaller
// keys of its records, one wave per 64 of them, writing each query's output
// segment as the radix sort's last pass does.  Work per bin grows with the
// square of its size, so it is chosen only for graphs with varied weights,
// and the ranking is bounded: when some bin holds more than kBucketRankMax
// records the layout launch sets ctl->resort, the ranking launch returns at
// once, and the caller sorts the scattered records (grouped by bin in
// recs[1]) with the radix sort instead (launch_sort_out, selected = 1).
constexpr uint32_t kMaxBins = 65536;
constexpr uint32_t kBucketRankMax = 4096;
inline size_t bucket_words(uint32_t nbins) { return 4 * static_cast<size_t>(nbins) + 1; }
// The ranking launch also publishes the call state (state_words words from
// state to state_map, as launch_publish does), which is final by then.
hipError_t launch_bucket_sort(const CallBuffers &b, rn_pair *out, unsigned long long user_cap, const uint32_t *state,
                              uint32_t *state_map, uint32_t state_words, hipStream_t s);

// Small sort, for calls of k-closest-pairs queries only whose k add up to at
// most kSmallSort / 2: one block sorts the selected records (recs[1]) in LDS
// as 64-bit (query, dist, u, v) keys (query bits qb, vertex bits vb, distance
// bits from the device) and writes the output as the radix sort's last pass
// does; one launch instead of the radix sort's two per digit.  More than
// kSmallSort records (ties at the bound) or a key wider than 63 bits set
// ctl->resort, and the caller runs the radix sort.  The same block first lays
// out the output (as launch_layout with selected = 1, which the caller then
// skips), and, as the call's last kernel, publishes the call state as
// launch_publish does (state_words words from state to state_map).
constexpr uint32_t kSmallSort = 4096;
hipError_t launch_sort_small(const CallBuffers &b, uint32_t qb, uint32_t vb, rn_pair *out, unsigned long long user_cap,
                             const uint32_t *state, uint32_t *state_map, uint32_t state_words, hipStream_t s);

}  // namespace rn
