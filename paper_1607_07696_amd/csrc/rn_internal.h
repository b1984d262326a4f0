// rn_internal.h -- types shared by the library's host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rn.h"

namespace rn {

constexpr uint32_t kInf = 0xFFFFFFFFu;     // unreachable / empty distance
constexpr uint32_t kMaxDist = 0xFFFFFFFEu; // largest representable distance

// Argument errors found on the device while staging a query (QueryCtl::err bits).
enum : uint32_t {
    kErrRange = 1u,    // an id outside [0, V)
    kErrDupR = 2u,     // a duplicate in R
    kErrDupS = 4u,     // a duplicate in S
    kErrOverlap = 8u,  // a vertex in both R and S
};

// Search tiers: up to three on-chip table sizes, then the global-memory tier
// that takes any search (novf[t] counts the sources re-run after tier t).
constexpr int kLdsTiers = 3;
constexpr int kTiers = kLdsTiers + 1;

// Device-resident control block of one query.  Zeroed before every query.
struct QueryCtl {
    uint32_t err;                   // kErr* bits
    uint32_t nsrc;                  // sources staged
    unsigned long long npairs;      // pairs emitted (may exceed the pair buffer)
    uint32_t novf[kTiers];          // sources that outgrew tier t (re-run at tier t+1)
    uint32_t theta;                 // k-closest pairs: current distance bound
    uint32_t ncand;                 // k-closest pairs: bound-seeding candidate count
    unsigned long long arcs;        // work count: out-arcs of every settled (source, vertex)
    unsigned long long settled;     // work count: settled (source, vertex) pairs
    unsigned long long nsel;        // k-closest pairs: candidates kept by the final bound
};

// k-closest pairs: distances are counted in log-spaced bins (16 per octave:
// exact below 16, then 16 steps per power of two); the upper edge of the bin
// holding the k-th count bounds the k-th smallest distance from above.
constexpr uint32_t kDistBins = 512;   // 464 used
static_assert(sizeof(QueryCtl) % 4 == 0, "QueryCtl is cleared as 32-bit words");

// One arc as the relaxation kernels read it: target, weight, and the target's
// own arc range, so expanding a vertex needs no separate row_ptr lookup.
struct alignas(16) ArcRec {
    int32_t y;
    uint32_t w;
    int32_t ybeg;
    int32_t yend;
};

// Arguments of one relaxation launch.
struct JoinArgs {
    const int32_t *row_ptr;     // [V+1]
    const ArcRec *arcs;         // [A]
    const uint32_t *sbits;      // S membership bitmap
    const int32_t *src;         // source vertex ids
    const uint32_t *nsrc;       // device count of src
    QueryCtl *ctl;
    rn_pair *pairs;             // emitted pairs
    unsigned long long pair_cap;
    uint32_t *ovf;              // sources that outgrew this tier (vertex ids)
    uint32_t *novf;             // device count of ovf
    uint32_t theta;             // bound for the theta-join
    uint32_t delta;             // bucket width (0 = one bucket)
    int32_t kcp;                // 1: bound is ctl->theta, read every phase
    int32_t count_work;         // 1: accumulate ctl->arcs / ctl->settled
    uint32_t k;                 // k-closest pairs: k
    uint32_t *cand_hist;        // k-closest pairs: kDistBins counts of emitted distances
};

// Per-source state of the global-memory tier, one slot per concurrent block:
// dist[V] | queued bitmap[ceil(V/32)] | frontier[V] | next frontier[V] | touched[V].
// Between searches dist is all kInf and the bitmap all zero.
inline size_t global_slot_words(int32_t V) {
    return 4 * static_cast<size_t>(V) + (static_cast<size_t>(V) + 31) / 32;
}

// Launchers (rn_kernels.hip).  All take the stream to enqueue on.
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_stage(const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, int32_t V,
                        const int32_t *rank, const int32_t *order, uint32_t *rbits,
                        uint32_t *sbits, int32_t *src, QueryCtl *ctl, uint32_t *scratch,
                        hipStream_t s);
size_t stage_scratch_words(int32_t V);
// Relaxation at table tier `tier` (log2 size hash_log2); grid chosen inside.
hipError_t launch_join(const JoinArgs &a, int hash_log2, uint32_t max_sources, hipStream_t s);
int join_tier_supported(int hash_log2);
// The global-memory tier: one block per source, nslots slots of
// global_slot_words(V) words each.
hipError_t launch_join_global(const JoinArgs &a, uint32_t *slots, uint32_t nslots, int32_t V,
                              uint32_t max_sources, hipStream_t s);
// Sort pairs[0 .. min(*n, cap)) by (dist, u, v) (scratch: another buffer of
// cap pairs) and write them to out when the query succeeded and the result
// fits (no argument error, no search left over, *n <= user_cap, *n <= cap).
// hist: sort_hist_words() words, zero on entry.  max_dist bounds every dist.
// Only the first out_limit sorted pairs are written (all of them for a theta-join).
hipError_t launch_sort_to_out(rn_pair *pairs, rn_pair *scratch, const unsigned long long *n,
                              unsigned long long cap, uint32_t max_dist, int32_t V, uint32_t *hist,
                              rn_pair *out, unsigned long long user_cap, unsigned long long out_limit,
                              const QueryCtl *ctl, int last_tier, hipStream_t s);
size_t sort_hist_words();
// k-closest pairs: seed the bound ctl->theta from the direct arcs between R and
// S (seed_hist: kDistBins zeroed words), then, after the searches, keep the
// emitted pairs within the final bound (into `kept`, count ctl->nsel).
hipError_t launch_kcp_seed(const int32_t *src, const uint32_t *nsrc, uint32_t max_sources,
                           const int32_t *row_ptr, const ArcRec *arcs, const uint32_t *sbits,
                           uint32_t *seed_hist, uint32_t k, QueryCtl *ctl, hipStream_t s);
hipError_t launch_kcp_filter(const rn_pair *pairs, unsigned long long cap, rn_pair *kept, QueryCtl *ctl,
                             hipStream_t s);
// Copy sorted pairs to the caller when the query succeeded and fits.
hipError_t launch_copy_out(const rn_pair *src, rn_pair *dst, const unsigned long long *n,
                           const QueryCtl *ctl, unsigned long long user_cap, unsigned long long limit,
                           unsigned long long out_limit, int last_tier, hipStream_t s);

}  // namespace rn
