// rn_kernels.hip -- gfx950 kernels of the network-distance joins.
//
// A call runs any mix of theta-joins and k-closest-pairs queries, each on one
// of the resident graphs, as one launch sequence on one HIP stream:
//   stage     validate every query's R and S, set its S-membership bitmap and
//             list all sources query by query (k_mark, k_overlap_count, k_rank_emit)
//   seed      k-closest pairs: a first distance bound per query from the
//             direct R-S arcs (k_kcp_seed_*); a query whose bound is below twice
//             the lightest arc is answered here, one thread per source (k_kcp_direct)
//   relax     one wavefront per source: a bounded, bucketed label-correcting
//             search whose whole state (distance table, pending set, frontier)
//             lives in LDS; emits (u, v, dist, query) for v in S (k_join), with
//             larger tables and a global-memory tier for searches that outgrow
//             the first
//   select    k-closest pairs: keep the records within the final bounds
//   sort      LSD radix sort of the records on the (query, dist, u, v) key;
//             the last digit pass writes each query's segment of the output
//
// The queries are the paper's theta-join and k-closest pairs (Abstract;
// Section 1; Section 4).  The per-source search plays the role of the paper's
// local best-first search from each w in R that tests every reached node for
// membership in S (Section 4, the text after Algorithm 3); here it is not
// confined to a partition, so no cross-edge expansion (Algorithms 3-4) is
// needed and the result is exact.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rn_internal.h"

namespace rn {

namespace {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // empty table key (vertex ids are below 2^31 - 1)
constexpr uint32_t kWin = 256;            // frontier arcs expanded per window (4 per lane)

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint32_t popc(uint64_t m) { return static_cast<uint32_t>(__popcll(m)); }

// Cross-lane move through DPP: lanes without a source (or masked off) get `identity`.
// Controls used: row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t v, uint32_t identity) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(identity), static_cast<int>(v),
                                                             CTRL, ROW_MASK, BANK_MASK, false));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), lane));
}

// Inclusive prefix sum over the 64 lanes: sums within 16-lane rows (shifts by
// 1, 2, 3, then 4 and 8 on the upper banks), then row totals carried across
// rows with the two row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    uint32_t s = v + dpp<0x111>(v, 0u);
    s += dpp<0x112>(v, 0u);
    s += dpp<0x113>(v, 0u);
    s += dpp<0x114, 0xf, 0xe>(s, 0u);
    s += dpp<0x118, 0xf, 0xc>(s, 0u);
    s += dpp<0x142, 0xa, 0xf>(s, 0u);
    s += dpp<0x143, 0xc, 0xf>(s, 0u);
    return s;
}

// Minimum over the 64 lanes, returned to every lane.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = min(v, dpp<0x111>(v, kInf));
    v = min(v, dpp<0x112>(v, kInf));
    v = min(v, dpp<0x114>(v, kInf));
    v = min(v, dpp<0x118>(v, kInf));
    v = min(v, dpp<0x142, 0xa, 0xf>(v, kInf));
    v = min(v, dpp<0x143, 0xc, 0xf>(v, kInf));
    return readlane(v, 63);
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Log-spaced distance bins (k-closest pairs): exact below 16, then 16 bins
// per power of two.
__device__ __forceinline__ uint32_t dist_bin(uint32_t d) {
    if (d < 16u) return d;
    const uint32_t e = 31u - static_cast<uint32_t>(__clz(d));   // e >= 4
    return 16u + (e - 4u) * 16u + ((d >> (e - 4u)) & 15u);
}

// Largest distance in bin b.
__device__ __forceinline__ uint32_t bin_upper(uint32_t b) {
    if (b < 16u) return b;
    const uint32_t e = (b - 16u) / 16u + 4u, m = (b - 16u) % 16u;
    const uint64_t u = ((16ull + m + 1ull) << (e - 4u)) - 1ull;
    return u > kMaxDist ? kMaxDist : static_cast<uint32_t>(u);
}

// Upper edge of the bin where the cumulative count of hist[0..kDistBins)
// reaches k (kMaxDist if the total is below k).  Called by a whole wave;
// result wave-uniform.  Counts read late only make the edge larger, so a
// stale read still yields an upper bound.
__device__ __forceinline__ uint32_t wave_bound_from_hist(const uint32_t *hist, uint32_t k) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint4 *p = reinterpret_cast<const uint4 *>(hist + 8u * lane);
    const uint4 x = p[0], y = p[1];
    const uint32_t c[8] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) sum += c[i];
    const uint32_t incl = wave_incl_scan(sum);
    if (readlane(incl, 63) < k) return kMaxDist;
    uint32_t run = incl - sum, found = kInf;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        run += c[i];
        if (found == kInf && run >= k) found = bin_upper(8u * lane + i);
    }
    return wave_min(found);
}

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    uint32_t s = a + b;
    return s < a ? kInf : s;
}

template <int HB>
__device__ __forceinline__ uint32_t slot_hash(uint32_t y) {
    return (y * 0x9E3779B1u) >> (32 - HB);
}

__device__ __forceinline__ uint32_t lds_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void lds_store(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// ------------------------------------------------------------------ per-source search state
// H: distance-table slots (open addressing, linear probing, filled to at most
// 3/4).  PC: capacity of each vertex list (pending set, frontier).  CT: the
// compact table (one 32-bit word per slot, below), else the wide one (a key
// array and a distance-word array).
template <int HB, bool CT>
struct Tier {
    static constexpr int H = 1 << HB;
    // list capacity: the ring (2 PC entries) holds a search's pending set (at
    // most about 120 vertices for searches that fit 2^11 entries on road
    // graphs, 250 for 2^13 and 370 for 2^14); sized so that every wide table
    // from 2^11 on fits 8 waves per CU.  The compact 2^11 search takes a ring
    // of 128 entries: 10 KiB in all, so 16 fit a CU instead of 14 (8% faster
    // on the 1024x1024 road graph at theta = 3000, where none of 8192 searches
    // outgrew it); a search that does goes on to the next tier.  Calls with delta > 0 take
    // the wide 2^11 table instead, whose lists of 128 entries their buckets need
    static constexpr int PC = (CT && HB == kCompactSmallRingHB) ? 64 : (HB <= 12 ? 128 : (HB == 13 ? 256 : 512));
    static constexpr int U = (H / 64) < 8 ? (H / 64) : 8;   // table rows scanned per batch
    // waves per search: a large table leaves room for few searches per CU, so
    // several waves share each one (a block): two for 2^12, four for 2^13,
    // eight for a wide 2^14 table (one search per CU) and three for a compact
    // one (two searches per CU fit the LDS); every wave takes 64 vertices per
    // step and has its own window of W arcs.  (More waves per search are
    // slower where the pending set is smaller than a step: eight on 2^13, two
    // on 2^11.)
    static constexpr int NW = HB >= 14 ? (CT ? 3 : 8) : (HB == 13 ? 4 : (HB == 12 ? 2 : 1));
    static constexpr int G = 1;
    static constexpr uint32_t W = kWin * G;
    // window map entries of 4 bytes (the lane expanding the arc's tail, and the
    // arc's index) instead of 8 (the arc's index and the tail's distance): the
    // compact 2^11 search then needs 11 KiB of LDS with a 256-entry ring (14
    // fit a CU instead of 12, 5% faster at theta = 3000) and 10 KiB with the
    // 128-entry ring it takes; at 2^10 the 8-byte form is faster (18 searches
    // per CU already), and the larger tables gain no residency
    static constexpr bool LW = CT && HB >= 11;
};

// Ring bookkeeping shared by the waves of a block that runs one search
// (tables of 2^12 entries and more).
struct BlockRing {
    uint32_t tail;      // unwrapped ring index of the next append (atomic)
    uint32_t nins;      // table entries in use (atomic)
    uint32_t ovf;       // the search outgrew this tier
    uint32_t dmin[2];   // least distance taken by the step, by step parity (atomic)
};

__device__ __forceinline__ uint32_t wave_in_block() { return threadIdx.x >> 6; }

// Distance words: (distance << 1) | pending, the low bit set while the vertex
// is in the pending list.  One atomicMin with (nd << 1) | 1 lowers the distance
// and marks the vertex pending only when nd is strictly smaller (an equal
// distance over a zero-weight arc leaves the word alone); the lane that finds
// the old word idle or empty appends the vertex.  Expansion clears the bit.
// Wide tables therefore hold distances up to 2^31 - 2; a search that needs
// longer ones moves on to the global tier.
constexpr uint32_t kWordNone = 0xFFFFFFFFu;   // empty slot (above every stored word)
constexpr uint32_t kPackMax = 0x7FFFFFFEu;    // largest distance a wide table holds
constexpr uint32_t kNoKey = 0xFFFFFFFEu;      // compare value no stored key (or compact word) equals

// Compact tables hold a slot's distance word and the identity of its vertex
// in one 32-bit word, which halves a search's LDS (8 KiB for 2^11 slots
// instead of 16) so that more searches fit a CU.  The vertex's local id y
// (below 2^24) is hashed by a bijection of 24-bit integers, z = y * kHash24 mod
// 2^24 (Fibonacci hashing); the top HB bits of z give the home slot, and a
// slot stores the other IDB = 24 - HB bits (the remainder) and the probe
// distance from the home slot (DB bits), which together with the slot
// determine z and so y.  Above them sits the distance word, (distance << 1) |
// pending, in the remaining HB + 5 bits:
//   [ distance | pending | probe distance | remainder ]
// Words of one vertex differ only in the distance word, so atomicMin on a
// slot known to hold the vertex acts as on the wide table's distance word,
// and a compare-and-swap on an empty slot claims it with its first distance.
// A search whose distance or probe sequence does not fit moves on to a
// wide table.
constexpr uint32_t kHash24 = 10368889u;       // odd, about 2^24 / golden ratio
constexpr uint32_t inverse_mod_2_32(uint32_t a) {
    uint32_t x = a;                            // Newton: each step doubles the correct low bits
    for (int i = 0; i < 5; ++i) x *= 2u - a * x;
    return x;
}
constexpr uint32_t kHash24Inv = inverse_mod_2_32(kHash24) & 0xFFFFFFu;
static_assert(((kHash24 * kHash24Inv) & 0xFFFFFFu) == 1u, "24-bit hash inverse");
static_assert(kCompactVertices == (1 << 24), "compact tables hash 24-bit local ids");

template <int HB>
struct Compact {
    static constexpr uint32_t IDB = 24u - HB;                 // remainder bits
    static constexpr uint32_t DB = compact_disp_bits(HB);     // probe distance bits
    static constexpr uint32_t SH = IDB + DB;                  // position of the distance word
    static constexpr uint32_t REM = (1u << IDB) - 1u;
    static constexpr uint32_t IDM = (1u << SH) - 1u;          // identity: probe distance and remainder
    static constexpr uint32_t PEND = 1u << SH;                // the pending bit
    static constexpr uint32_t MAXP = (1u << DB) - 1u;         // longest probe distance
    // largest distance: its word stays below kNoKey and kWordNone
    static constexpr uint32_t MAXD = compact_max_dist(HB);
    static_assert(((((MAXD << 1) | 1u) << SH) | IDM) < kNoKey, "a compact word never equals kNoKey");
};

__device__ __forceinline__ uint32_t hash24(uint32_t y) { return (y * kHash24) & 0xFFFFFFu; }

template <int HB, bool CT>
struct SearchLds;

template <int HB>
struct SearchLds<HB, false> {
    static constexpr int H = Tier<HB, false>::H;
    static constexpr int PC = Tier<HB, false>::PC;
    uint32_t key[H];            // vertex id (global), or kEmpty
    uint32_t dw[H];             // distance word, kWordNone when empty
    uint2 lst[2][PC];           // two vertex lists of {slot | (arc count << 16), first arc} (with
                                //   delta = 0, one ring of 2 PC entries over the same words)
    uint2 win[Tier<HB, false>::W * Tier<HB, false>::NW];   // per wave: window arc -> {arc index,
                                //   distance of the arc's tail}; outside a window step, entry
                                //   lane is the write sink of lanes with nothing to store
                                //   (distinct addresses, no serialised writes) and the staging
                                //   area of emitted pairs
    __device__ uint2 *wwin() {
        if constexpr (Tier<HB, false>::NW == 1) return win;
        else return win + wave_in_block() * Tier<HB, false>::W;
    }
    __device__ uint2 *sink() { return wwin() + lane_id(); }
};

template <int HB>
struct SearchLds<HB, true> {
    static constexpr int H = Tier<HB, true>::H;
    static constexpr int PC = Tier<HB, true>::PC;
    uint32_t t[H];              // compact word, kWordNone when empty
    uint2 lst[2][PC];           // as in the wide table
    using WinEntry = std::conditional_t<Tier<HB, true>::LW, uint32_t, uint2>;
    WinEntry win[Tier<HB, true>::W * Tier<HB, true>::NW];   // per wave: as in the wide table, or
                                //   (Tier::LW) window arc -> (lane holding its tail << 26) | arc
                                //   index (below 2^26), the tail's distance coming over the lanes
    __device__ WinEntry *wwin() {
        if constexpr (Tier<HB, true>::NW == 1) return win;
        else return win + wave_in_block() * Tier<HB, true>::W;
    }
    __device__ uint2 *sink() { return reinterpret_cast<uint2 *>(wwin()) + lane_id(); }
};

// ---- table access shared by both layouts
// Distance held in slot s.
template <int HB, bool CT>
__device__ __forceinline__ uint32_t slot_dist(SearchLds<HB, CT> &L, uint32_t s) {
    if constexpr (CT) return L.t[s] >> (Compact<HB>::SH + 1u);
    else return L.dw[s] >> 1;
}

// Clear the pending bit of slot s (lanes with !valid issue a no-op on their own slot).
template <int HB, bool CT>
__device__ __forceinline__ void clear_pending(SearchLds<HB, CT> &L, uint32_t s, bool valid) {
    if constexpr (CT) atomicAnd(&L.t[valid ? s : lane_id()], valid ? ~Compact<HB>::PEND : 0xFFFFFFFFu);
    else atomicAnd(&L.dw[valid ? s : lane_id()], valid ? ~1u : 0xFFFFFFFFu);
}

// Set slot s pending again; returns whether it already was.
template <int HB, bool CT>
__device__ __forceinline__ bool mark_pending(SearchLds<HB, CT> &L, uint32_t s, bool valid) {
    if constexpr (CT)
        return (atomicOr(&L.t[valid ? s : lane_id()], valid ? Compact<HB>::PEND : 0u) & Compact<HB>::PEND) != 0u;
    else
        return (atomicOr(&L.dw[valid ? s : lane_id()], valid ? 1u : 0u) & 1u) != 0u;
}

// Empty slot s.
template <int HB, bool CT>
__device__ __forceinline__ void clear_slot(SearchLds<HB, CT> &L, uint32_t s) {
    if constexpr (CT) {
        lds_store(&L.t[s], kWordNone);
    } else {
        lds_store(&L.key[s], kEmpty);
        L.dw[s] = kWordNone;
    }
}

// Vertex (global id) and distance in slot s; false if the slot is empty.
template <int HB, bool CT>
__device__ __forceinline__ bool read_slot(SearchLds<HB, CT> &L, uint32_t s, int32_t voff, uint32_t &y,
                                          uint32_t &d) {
    if constexpr (CT) {
        using K = Compact<HB>;
        const uint32_t w = lds_load(&L.t[s]);
        const uint32_t home = (s - ((w >> K::IDB) & K::MAXP)) & (Tier<HB, true>::H - 1u);
        y = ((((home << K::IDB) | (w & K::REM)) * kHash24Inv) & 0xFFFFFFu) + static_cast<uint32_t>(voff);
        d = w >> (K::SH + 1u);
        return w != kWordNone;
    } else {
        y = lds_load(&L.key[s]);
        d = L.dw[s] >> 1;
        return y != kEmpty;
    }
}

// Put source u (global id) at distance 0, pending, into the empty table;
// returns its slot.
template <int HB, bool CT>
__device__ __forceinline__ uint32_t put_source(SearchLds<HB, CT> &L, int32_t u, int32_t voff) {
    if constexpr (CT) {
        using K = Compact<HB>;
        const uint32_t z = hash24(static_cast<uint32_t>(u - voff));
        const uint32_t h0 = z >> K::IDB;
        lds_store(&L.t[h0], K::PEND | (z & K::REM));
        return h0;
    } else {
        const uint32_t h0 = slot_hash<HB>(static_cast<uint32_t>(u));
        lds_store(&L.key[h0], static_cast<uint32_t>(u));
        L.dw[h0] = 1u;
        return h0;
    }
}

struct WaveState {
    uint32_t np;    // entries queued (pending list, or the ring between head and tail)
    uint32_t tail;  // flat list index of the next append (ring: unwrapped counter)
    uint32_t amask; // append index mask (ring: its size - 1; pending list: all ones)
    uint32_t cap;   // most entries the queue may hold
    uint32_t nins;  // table entries in use
    uint32_t imin;  // per-lane min of the distances improved this phase
    uint32_t pnew;  // k-closest pairs: discoveries counted this phase, not yet published
    bool ovf;       // the search outgrew this tier
    bool probing;   // k-closest pairs: count discoveries of S members
    uint32_t head;  // block search: the ring's head once this step's entries are taken
    BlockRing *blk; // block search: the shared ring state (else null)
};

// What a search needs to know about its query (read once per source; uniform
// across the wave, so the compiler keeps it in scalar registers).
struct SrcCtx {
    uint32_t theta;                 // the query's own bound
    uint32_t k;                     // 0: theta-join
    uint32_t delta;
    int32_t voff;                   // first global id of the query's graph
    uint32_t q;
    uint32_t tier;
    uint32_t rpo;                   // row pointer offset of the arcs searched
    uint32_t wmin;                  // lightest arc weight of the graph
    uint32_t slack;                 // delta = 0: how far above a step's least distance a vertex waits
    bool swapped;                   // the search runs from S: emitted pairs are reversed
    bool big_deg;                   // some vertex of the graph has 2^16 or more arcs
    const uint32_t *sbits;          // the query's S bitmap (local ids)
    uint32_t *hist;                 // k > 0: the query's histogram region (else null)
    QueryState *qs;                 // the query's state
};

__device__ __forceinline__ SrcCtx load_ctx(const JoinArgs &a, uint32_t q) {
    const QueryDesc &d = a.qd[q];
    SrcCtx c;
    c.theta = d.theta;
    c.k = d.k;
    c.delta = d.delta;
    c.voff = d.voff;
    c.q = q;
    c.tier = static_cast<uint32_t>(a.tier);
    c.rpo = d.orient & ~kOrientSwap;
    c.wmin = d.wmin;
    c.slack = d.slack;
    c.swapped = (d.orient & kOrientSwap) != 0;
    c.big_deg = a.big_deg != 0;
    c.sbits = a.sbits + d.sbits;
    c.hist = d.k ? a.hists + d.hist : nullptr;
    c.qs = a.qs + q;
    return c;
}

__device__ __forceinline__ uint32_t *probe_hist(const SrcCtx &c) { return c.hist + kHistProbe + c.tier * kDistBins; }
__device__ __forceinline__ uint32_t *probe_count(const SrcCtx &c) { return c.hist + kHistCount + c.tier; }

__device__ __forceinline__ uint32_t current_bound(const SrcCtx &c) {
    if (c.k == 0) return c.theta;
    const uint32_t t = __hip_atomic_load(&c.qs->bound, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return min(t, c.theta);
}

__device__ __forceinline__ bool in_s(const SrcCtx &c, uint32_t y) {
    const uint32_t yl = y - static_cast<uint32_t>(c.voff);
    return (c.sbits[yl >> 5] >> (yl & 31u)) & 1u;
}

// Whether arc x is the first lightest of the arcs joining its tail to its
// target: parallel arcs make one pair, at the lightest weight (bits computed
// on the host when the graph is uploaded).
__device__ __forceinline__ bool first_of_pair(const JoinArgs &a, int32_t x) {
    return (a.first[static_cast<uint32_t>(x) >> 5] >> (x & 31)) & 1u;
}

// The caller's local id of global vertex x of the device copy (which
// rn_partition renumbers in leaf order).
__device__ __forceinline__ int32_t caller_id(const JoinArgs &a, int32_t x, int32_t voff) {
    return a.order ? a.order[x] : x - voff;
}

// Discoveries a query's searches count per tier before they stop: enough for
// a close bound, few enough to keep the histogram atomics cheap.
__device__ __forceinline__ uint32_t probe_cap(const SrcCtx &c) { return max(4u * c.k, 256u); }

// k-closest pairs, at the start of a phase: publish the discoveries of the
// last phase, lower the shared bound from this tier's discovery histogram
// once it holds k pairs (and again each time it has grown by an eighth), and
// decide whether to keep counting.  Whole wave; the result is wave-uniform.
__device__ __forceinline__ void probe_phase(const SrcCtx &c, uint32_t &pnew, bool &probing, uint32_t &seen) {
    uint32_t *cnt = probe_count(c);
    uint32_t n = 0;
    if (lane_id() == 0)
        n = pnew ? atomicAdd(cnt, pnew) + pnew : __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    n = readlane(n, 0);
    pnew = 0;
    probing = n < probe_cap(c);
    if (n < c.k || n < seen + (seen >> 3) + 1u) return;
    seen = n;
    const uint32_t b = wave_bound_from_hist(probe_hist(c), c.k);
    if (lane_id() == 0) atomicMin(&c.qs->bound, b);
}

// Relax NJ window arcs per lane (slot j holds window arc j*64 + lane) and
// append targets that became pending to list P.  Two LDS steps, each issued
// for all NJ slots before any result is used: claim-or-find the target's slot
// (compare-and-swap on an empty home slot doubles as the first probe), then
// the packed atomicMin.  Idle lanes issue no-op atomics instead of branching.
// Called by all 64 lanes; st.ovf is wave-uniform afterwards.
template <int HB, bool CT, int NJ>
__device__ __forceinline__ void relax_window(SearchLds<HB, CT> &L, WaveState &st, const SrcCtx &c,
                                             const ArcRec *r, const uint32_t *nd, uint32_t bound) {
    constexpr uint32_t H = Tier<HB, CT>::H;
    // slot states: 0 idle, 1 slot holds y, 2 slot claimed for y, 3 keep probing;
    // after the min, flags: the distance improved (imp), and the vertex was
    // idle or new, so this lane appends it (app)
    uint32_t h[NJ], stt[NJ], old[NJ];
    bool fresh[NJ];   // the slot was empty before this window: a new table entry
    bool app[NJ];     // this lane appends the vertex (it was idle or new, and improved)
    bool imp[NJ];     // the vertex's distance improved
    // a distance the table's word cannot hold (possible only when the bound
    // itself is that large) sends the search on to the next tier
    constexpr uint32_t kMaxWord = CT ? Compact<HB>::MAXD : kPackMax;
    const uint32_t lim = min(bound, kMaxWord);
    bool lost = false;
    if (bound > kMaxWord) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) lost |= nd[j] <= bound && nd[j] > kMaxWord;
    }
    if constexpr (CT) {
        using K = Compact<HB>;
        // compare-and-swap of the vertex's word (distance nd, pending, probe
        // distance 0) into its home slot: an empty slot is claimed with its
        // first distance at once; a slot of the same identity holds y (then
        // the atomicMin below); any other identity sends y one slot on
        uint32_t nw[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const bool act = nd[j] <= lim;
            const uint32_t z = hash24(static_cast<uint32_t>(r[j].y - c.voff));
            // idle lanes aim their no-op atomics at distinct slots: a shared address would serialise
            h[j] = act ? z >> K::IDB : lane_id();
            nw[j] = act ? ((((nd[j] << 1) | 1u) << K::SH) | (z & K::REM)) : kWordNone;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) old[j] = atomicCAS(&L.t[h[j]], nd[j] <= lim ? kWordNone : kNoKey, nw[j]);
        __builtin_amdgcn_sched_barrier(0);   // every claim is issued before the first result is used
        bool probe = false;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            stt[j] = nd[j] > lim ? 0u : (old[j] == kWordNone ? 2u : (((old[j] ^ nw[j]) & K::IDM) == 0u ? 1u : 3u));
            probe |= stt[j] == 3u;
        }
        if (__ballot(probe) != 0) {
            // linear probing in rounds, as in the wide table; the probe
            // distance is part of the identity, so it is raised with the slot
            for (uint32_t round = 1;; ++round) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const bool act = stt[j] == 3u;
                    h[j] = act ? ((h[j] + 1u) & (H - 1)) : h[j];
                    nw[j] += act ? (1u << K::IDB) : 0u;
                    old[j] = atomicCAS(&L.t[act ? h[j] : lane_id()], act ? kWordNone : kNoKey, nw[j]);
                }
                bool more = false;
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    if (stt[j] == 3u)
                        stt[j] = old[j] == kWordNone ? 2u : (((old[j] ^ nw[j]) & K::IDM) == 0u ? 1u : 3u);
                    more |= stt[j] == 3u;
                }
                if (__ballot(more) == 0) break;
                if (round >= K::MAXP) {   // the probe distance field is full
                    lost = lost || more;
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        nw[j] = stt[j] == 3u ? kWordNone : nw[j];
                        stt[j] = stt[j] == 3u ? 0u : stt[j];
                    }
                    break;
                }
            }
        }
        // the min on slots found to hold y; claimed slots already hold nd
#pragma unroll
        for (int j = 0; j < NJ; ++j) old[j] = atomicMin(&L.t[stt[j] == 1u ? h[j] : lane_id()], stt[j] == 1u ? nw[j] : kWordNone);
        __builtin_amdgcn_sched_barrier(0);   // every min is issued before the first result is used
        // a claimed slot compares as a word above every word a vertex can
        // hold, and not pending: the vertex counts as improved and is
        // appended by the claiming lane.  Idle lanes carry kWordNone, which
        // compares above nothing.
        constexpr uint32_t kClaimed = ~K::PEND;
        static_assert(((((K::MAXD << 1) | 1u) << K::SH) | K::IDM) < kClaimed, "a claimed slot compares above every word");
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            fresh[j] = stt[j] == 2u;
            const uint32_t o = fresh[j] ? kClaimed : old[j];
            imp[j] = nw[j] < o;
            // the vertex is appended if it improved and was idle: a pending
            // old word is cut to the bits below its pending bit, which every
            // word exceeds, so that one comparison decides
            app[j] = nw[j] < (o & ((o & K::PEND) - 1u));
        }
    } else {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            // idle lanes aim their no-op atomics at distinct slots: a shared address would serialise
            h[j] = nd[j] <= lim ? slot_hash<HB>(static_cast<uint32_t>(r[j].y)) : lane_id();
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            old[j] = atomicCAS(&L.key[h[j]], nd[j] <= lim ? kEmpty : kNoKey, static_cast<uint32_t>(r[j].y));
        __builtin_amdgcn_sched_barrier(0);   // every claim is issued before the first result is used
        bool probe = false;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const uint32_t y = static_cast<uint32_t>(r[j].y);
            stt[j] = nd[j] > lim ? 0u : (old[j] == kEmpty ? 2u : (old[j] == y ? 1u : 3u));
            probe |= stt[j] == 3u;
        }
        if (__ballot(probe) != 0) {
            // linear probing past an occupied home slot, in rounds: each round
            // moves every slot still searching one place on and issues all their
            // compare-and-swaps (no-ops for the rest) before any result is used.
            // (Linear probing beats double hashing here: the ids of a ball are
            // clustered, and multiplicative hashing spreads runs of them evenly.)
            for (uint32_t round = 1;; ++round) {
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const bool act = stt[j] == 3u;
                    h[j] = act ? ((h[j] + 1u) & (H - 1)) : h[j];
                    old[j] = atomicCAS(&L.key[act ? h[j] : lane_id()], act ? kEmpty : kNoKey,
                                       static_cast<uint32_t>(r[j].y));
                }
                bool more = false;
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const uint32_t y = static_cast<uint32_t>(r[j].y);
                    if (stt[j] == 3u) stt[j] = old[j] == kEmpty ? 2u : (old[j] == y ? 1u : 3u);
                    more |= stt[j] == 3u;
                }
                if (__ballot(more) == 0) break;
                if (round >= H) {   // every slot visited: the table is full
                    lost = lost || more;
                    break;
                }
            }
        }
        uint32_t v[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            v[j] = (stt[j] == 1u || stt[j] == 2u) ? (nd[j] << 1) | 1u : kWordNone;   // nd <= lim here
            old[j] = atomicMin(&L.dw[h[j]], v[j]);
        }
        __builtin_amdgcn_sched_barrier(0);   // every min is issued before the first result is used
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            imp[j] = v[j] < old[j];
            app[j] = imp[j] && (old[j] == kWordNone || (old[j] & 1u) == 0u);
            fresh[j] = imp[j] && old[j] == kWordNone;
        }
    }
    uint64_t mA[NJ];
    uint32_t nadd = 0, ins = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        st.imin = min(st.imin, imp[j] ? nd[j] : kInf);
        mA[j] = __ballot(app[j]);
        nadd += popc(mA[j]);
        ins += popc(__ballot(fresh[j]));
    }
    if (c.big_deg) {   // list entries hold arc counts below 2^16
#pragma unroll
        for (int j = 0; j < NJ; ++j) lost |= app[j] && (r[j].yend - r[j].ybeg) > 0xFFFF;
    }
    if constexpr (Tier<HB, CT>::NW == 1) st.nins += ins;
    if (st.probing && ins != 0) {
        // k-closest pairs: a first discovery of an S member is a pair with a
        // path of length nd
        uint32_t *ph = probe_hist(c);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const bool found = fresh[j] && in_s(c, static_cast<uint32_t>(r[j].y));
            if (found) atomicAdd(&ph[dist_bin(nd[j])], 1u);
            st.pnew += popc(__ballot(found));
        }
    }
    uint2 *q = &L.lst[0][0];
    if constexpr (Tier<HB, CT>::NW > 1) {
        // a block search: reserve ring entries and count table entries in
        // the block's shared state (one atomic each per wave)
        uint32_t base = 0, fill = 0;
        if (lane_id() == 0) {
            base = atomicAdd(&st.blk->tail, nadd);
            fill = atomicAdd(&st.blk->nins, ins) + ins;
        }
        base = readlane(base, 0);
        fill = readlane(fill, 0);
        if (__ballot(lost) != 0 || fill > (3u * H) / 4u || base + nadd - st.head > st.cap) {
            st.ovf = true;
            if (lane_id() == 0) st.blk->ovf = 1u;
            return;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            uint2 *dst = app[j] ? q + ((base + mbcnt(mA[j])) & st.amask) : L.sink();
            *dst = make_uint2(h[j] | (static_cast<uint32_t>(r[j].yend - r[j].ybeg) << 16),
                              static_cast<uint32_t>(r[j].ybeg));
            base += popc(mA[j]);
        }
        return;
    }
    if (__ballot(lost) != 0 || st.nins > (3u * H) / 4u || st.np + nadd > st.cap) {
        st.ovf = true;
        return;
    }
    uint32_t base = st.tail;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        uint2 *dst = app[j] ? q + ((base + mbcnt(mA[j])) & st.amask) : L.sink();
        *dst = make_uint2(h[j] | (static_cast<uint32_t>(r[j].yend - r[j].ybeg) << 16),
                          static_cast<uint32_t>(r[j].ybeg));
        base += popc(mA[j]);
    }
    st.np += base - st.tail;
    st.tail = base;
}

// Load window arcs j*64 + lane (j < NJ) and relax them.  Every load is issued
// before any is used; lanes past the window's end load arc 0 and stay idle.
// 4-byte window entries (Tier::LW) name the lane expanding the arc's tail,
// whose distance d0 comes over the lanes (ds_bpermute) while the arc loads run.
template <int HB, bool CT, int NJ>
__device__ __forceinline__ void window_step(SearchLds<HB, CT> &L, WaveState &st, const SrcCtx &c,
                                            const ArcRec *__restrict__ arcs, uint32_t cnt,
                                            uint32_t bound, uint32_t d0) {
    const uint32_t lane = lane_id();
    int32_t idx[NJ];
    uint32_t od[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint32_t t = j * 64 + lane;
        const uint32_t tc = t < cnt ? t : 0u;
        if constexpr (Tier<HB, CT>::LW) {
            const uint32_t e = L.wwin()[tc];
            idx[j] = t < cnt ? static_cast<int32_t>(e & (kCompactArcs - 1)) : 0;
            od[j] = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(static_cast<int>((e >> 26) << 2),
                                                                       static_cast<int>(d0)));
        } else {
            const uint2 w = L.wwin()[tc];
            idx[j] = t < cnt ? static_cast<int32_t>(w.x) : 0;
            od[j] = w.y;
        }
    }
    ArcRec r[NJ];
    uint32_t nd[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) r[j] = arcs[idx[j]];
    // (idle lanes: all ones, by a mask rather than a branch, so that no load is deferred)
#pragma unroll
    for (int j = 0; j < NJ; ++j) nd[j] = sat_add(od[j], r[j].w) | (j * 64 + lane < cnt ? 0u : kInf);
    wave_sync();  // window map fully read before the next window rewrites it
    relax_window<HB, CT, NJ>(L, st, c, r, nd, bound);
}

// k-closest pairs: once the query has emitted k records, bound its k-th
// distance by its emitted-distance histogram and lower the shared bound.
// Whole wave.
// seen: the count at this wave's last recomputation for the query; the bound
// is recomputed only once the count has grown by an eighth since then.
__device__ __forceinline__ void tighten_bound(const SrcCtx &c, unsigned long long &seen) {
    const unsigned long long n = __hip_atomic_load(&c.qs->npairs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n < c.k || n < seen + (seen >> 3) + 1ull) return;
    seen = n;
    const uint32_t b = wave_bound_from_hist(c.hist + kHistEmit, c.k);
    if ((threadIdx.x & 63u) == 0) atomicMin(&c.qs->bound, b);
}

// Reserve n record slots for query c (one atomic per wave); the base is
// returned to every lane.
__device__ __forceinline__ unsigned long long reserve_recs(const JoinArgs &a, const SrcCtx &c, uint32_t n) {
    unsigned long long base = 0;
    if (lane_id() == 0) {
        base = atomicAdd(&a.ctl->npairs, static_cast<unsigned long long>(n));
        atomicAdd(&c.qs->npairs, static_cast<unsigned long long>(n));
    }
    return (static_cast<unsigned long long>(readlane(static_cast<uint32_t>(base >> 32), 0)) << 32) |
           readlane(static_cast<uint32_t>(base), 0);
}

// theta-join calls sorted by bins: a record's place among its (query, dist)
// bin's records, from the bin count it was added to, is kept in the upper 16
// bits of its query field (queries are numbered below 2^16) until the scatter
// moves it; places of kPlaceNone and more are stored as kPlaceNone.
constexpr uint32_t kPlaceNone = 0xFFFFu;
static_assert(kMaxQueries <= 0x10000, "query numbers fit the low 16 bits of a record's query field");
__device__ __forceinline__ uint32_t bin_place(uint32_t place) { return min(place, kPlaceNone) << 16; }

// Write this wave's staged pairs ({dist, v} in stg) for source u.
template <int HB, bool CT>
__device__ __forceinline__ void flush_pairs(SearchLds<HB, CT> &L, const JoinArgs &a, const SrcCtx &c, int32_t u,
                                            uint32_t &nst, const uint2 *stg) {
    if (nst == 0) return;
    const unsigned long long base = reserve_recs(a, c, nst);
    const uint32_t bin0 = a.bins ? a.binbase[c.q] : 0u;
    wave_sync();
    for (uint32_t i = lane_id(); i < nst; i += 64) {
        const unsigned long long idx = base + i;
        if (idx < a.rec_cap) {
            Rec r;
            const uint2 e = stg[i];
            const int32_t from = caller_id(a, u, c.voff), to = caller_id(a, static_cast<int32_t>(e.y), c.voff);
            r.u = c.swapped ? to : from;
            r.v = c.swapped ? from : to;
            r.d = e.x;
            r.q = c.q;
            if (a.bins) r.q |= bin_place(atomicAdd(&a.bins[bin0 + r.d], 1u));
            a.recs[idx] = r;
        }
    }
    wave_sync();
    nst = 0;
}

// Expand up to 64 G queued vertices (G per lane: list entries eb[g], valid[g],
// distances d[g] read from the table just before, so that improvements made
// since a vertex was queued are used): clear their pending flags (unless the
// caller has: CLR = false), then relax their arcs, windows of 256 G at a
// time.  Whole wave.
template <int HB, bool CT, int G, bool CLR = true>
__device__ __forceinline__ void expand_chunk(SearchLds<HB, CT> &L, WaveState &st, const SrcCtx &c, const JoinArgs &a,
                                             const uint2 *eb, const bool *valid, const uint32_t *d,
                                             uint32_t bound) {
    constexpr uint32_t W = kWin * G;
    static_assert(!Tier<HB, CT>::LW || G == 1, "4-byte window entries name the expanding lane, one vertex per lane");
    static_assert(W * sizeof(uint32_t) >= 64 * sizeof(uint2), "the window area holds the wave's sink");
    uint32_t deg[G];
    int32_t b[G];
    uint32_t sum = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t e = eb[g].x;
        const uint32_t sl = e & 0xFFFFu;
        b[g] = static_cast<int32_t>(eb[g].y);
        if constexpr (CLR) clear_pending(L, sl, valid[g]);   // expanded now: not pending
        deg[g] = (valid[g] && d[g] <= bound) ? (e >> 16) : 0u;
        sum += deg[g];
    }
    const uint32_t incl = wave_incl_scan(sum);
    const uint32_t total = readlane(incl, 63);
    for (uint32_t wb = 0; wb < total && !st.ovf; wb += W) {
        uint32_t first = incl - sum;   // this lane's entries occupy [first, incl) in order
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t lo = max(first, wb), hi = min(first + deg[g], wb + W);
            for (uint32_t p = lo; p < hi; ++p) {
                if constexpr (Tier<HB, CT>::LW) L.wwin()[p - wb] = (lane_id() << 26) | (static_cast<uint32_t>(b[g]) + (p - first));
                else L.wwin()[p - wb] = make_uint2(static_cast<uint32_t>(b[g]) + (p - first), d[g]);
            }
            first += deg[g];
        }
        wave_sync();
        const uint32_t cnt = min(W, total - wb);
        switch ((cnt + 63u) / 64u) {
            case 1: window_step<HB, CT, 1>(L, st, c, a.arcs, cnt, bound, d[0]); break;
            case 2: window_step<HB, CT, 2>(L, st, c, a.arcs, cnt, bound, d[0]); break;
            case 3: window_step<HB, CT, 3>(L, st, c, a.arcs, cnt, bound, d[0]); break;
            case 4: window_step<HB, CT, 4>(L, st, c, a.arcs, cnt, bound, d[0]); break;
            default:
                if constexpr (G > 1) {
                    switch ((cnt + 63u) / 64u) {
                        case 5: window_step<HB, CT, 5>(L, st, c, a.arcs, cnt, bound, d[0]); break;
                        case 6: window_step<HB, CT, 6>(L, st, c, a.arcs, cnt, bound, d[0]); break;
                        case 7: window_step<HB, CT, 7>(L, st, c, a.arcs, cnt, bound, d[0]); break;
                        default: window_step<HB, CT, 8>(L, st, c, a.arcs, cnt, bound, d[0]); break;
                    }
                }
                break;
        }
        wave_sync();
    }
}

// k-closest pairs with a bound below twice the lightest arc: every path of two
// or more arcs is longer than the bound, so the pairs within it are exactly
// the direct arcs from u into S no heavier than the bound, at the weight of
// the lightest arc of each pair (parallel arcs: the first lightest).  The
// source emits those without a search.  Whole wave.
template <int HB, bool CT>
__device__ __forceinline__ void direct_pairs(SearchLds<HB, CT> &L, const JoinArgs &a, const SrcCtx &c, int32_t u,
                                             unsigned long long &tseen) {
    constexpr uint32_t PC = Tier<HB, CT>::PC;
    const uint32_t lane = lane_id();
    const uint32_t bound = current_bound(c);
    const int32_t ub = a.row_ptr[c.rpo + u], ue = a.row_ptr[c.rpo + u + 1];
    uint2 *const stg = &L.lst[0][0];   // both lists, 2 PC entries: free, no search runs
    uint32_t nst = 0, emitted = 0;
    for (int32_t x0 = ub; x0 < ue; x0 += 64) {
        const int32_t x = x0 + static_cast<int32_t>(lane);
        bool m = false;
        ArcRec r{0, 0, 0, 0};
        if (x < ue) {
            r = a.arcs[x];
            m = r.w <= bound && first_of_pair(a, x) && in_s(c, static_cast<uint32_t>(r.y));
        }
        const uint64_t mM = __ballot(m);
        if (m) atomicAdd(&c.hist[kHistEmit + dist_bin(r.w)], 1u);
        emitted += popc(mM);
        *(m ? stg + nst + mbcnt(mM) : L.sink()) = make_uint2(r.w, static_cast<uint32_t>(r.y));
        nst += popc(mM);
        if (nst + 64 > 2u * PC) {
            wave_sync();
            flush_pairs<HB, CT>(L, a, c, u, nst, stg);
        }
    }
    wave_sync();
    flush_pairs<HB, CT>(L, a, c, u, nst, stg);
    if (emitted != 0) tighten_bound(c, tseen);
    wave_sync();
}

// Bounded search from u.  Bucket b holds tentative distances in
// [b*delta, (b+1)*delta); each phase expands every pending vertex of the
// lowest non-empty bucket and relaxes its arcs.  With delta <= the smallest
// arc weight each vertex is expanded once, at its final distance (Dijkstra
// order by buckets); a larger delta trades re-expansions for fewer phases.
// delta = 0 has no buckets at all: the pending list is a FIFO ring, each step
// expands the 64 oldest pending vertices, and the vertices they improve queue
// up behind the rest at once, so no window waits for a phase to end.  The
// search ends when nothing is pending; every table entry then holds its exact
// distance, and entries in S become pairs.
template <int HB, bool CT>
__device__ void search_source(SearchLds<HB, CT> &L, const JoinArgs &a, const SrcCtx &c, int32_t u,
                              unsigned long long &tseen) {
    constexpr int H = Tier<HB, CT>::H;
    constexpr int PC = Tier<HB, CT>::PC;
    constexpr int U = Tier<HB, CT>::U;
    const uint32_t lane = lane_id();
    const int32_t ub = a.row_ptr[c.rpo + u];
    const int32_t ue = a.row_ptr[c.rpo + u + 1];
    if (lane == 0) {
        const uint32_t h0 = put_source(L, u, c.voff);   // the table is empty
        L.lst[0][0] = make_uint2(h0 | (static_cast<uint32_t>(min(ue - ub, 0xFFFF)) << 16), static_cast<uint32_t>(ub));
    }
    wave_sync();
    WaveState st;
    st.np = 1;
    st.nins = 1;
    st.pnew = 0;
    st.imin = kInf;
    st.ovf = (ue - ub) > 0xFFFF;
    st.probing = false;
    st.head = 0;
    st.blk = nullptr;
    uint32_t bound = c.theta;
    uint32_t seen = 0, phase = 0;

    if (c.delta == 0) {
        // one bucket: a FIFO ring of pending vertices; each step expands up to
        // 64 of them, and vertices they improve join the ring at once
        constexpr uint32_t RC = 2u * PC;
        uint2 *q = &L.lst[0][0];
        st.tail = 1;
        st.amask = RC - 1u;
        st.cap = RC;
        uint32_t head = 0;
        while (st.np > 0 && !st.ovf) {
            // small searches (the first two steps) never count discoveries
            if (c.hist != nullptr && phase >= 2) probe_phase(c, st.pnew, st.probing, seen);
            ++phase;
            bound = current_bound(c);
            constexpr int G = Tier<HB, CT>::G;
            const uint32_t m = min(64u * G, st.np);
            uint2 eb[G];
            bool valid[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                valid[g] = g * 64u + lane < m;
                eb[g] = q[(head + g * 64u + lane) & (RC - 1u)];
            }
            head += m;
            st.np -= m;
            wave_sync();  // the taken entries are read before appends reuse their slots
            uint32_t dd[G];
#pragma unroll
            for (int g = 0; g < G; ++g) dd[g] = slot_dist(L, valid[g] ? (eb[g].x & 0xFFFFu) : lane);
            if (c.slack != kInf) {
                // a vertex far above the step's least distance goes back to
                // the tail, still pending: its distance is likely to improve
                // before it comes round again, which saves expanding it twice
                uint32_t mn = kInf;
#pragma unroll
                for (int g = 0; g < G; ++g) mn = min(mn, valid[g] ? dd[g] : kInf);
                const uint32_t lim = sat_add(wave_min(mn), c.slack);
                uint32_t base = st.tail;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const bool later = valid[g] && dd[g] > lim && dd[g] <= bound;
                    const uint64_t mL = __ballot(later);
                    if (mL != 0) {   // (wave-uniform)
                        *(later ? q + ((base + mbcnt(mL)) & (RC - 1u)) : L.sink()) = eb[g];
                        base += popc(mL);
                        valid[g] = valid[g] && !later;
                    }
                }
                st.np += base - st.tail;
                st.tail = base;
            }
            expand_chunk<HB, CT, G>(L, st, c, a, eb, valid, dd, bound);
        }
    } else {
        uint32_t P = 0;      // list receiving appends (the pending list)
        uint32_t pmin = 0;
        while (st.np > 0 && !st.ovf) {
            if (c.hist != nullptr && phase >= 2) probe_phase(c, st.pnew, st.probing, seen);
            ++phase;
            bound = current_bound(c);
            const uint64_t t64 = (static_cast<uint64_t>(pmin / c.delta) + 1ull) * c.delta;
            const uint32_t thr = t64 > kInf ? kInf : static_cast<uint32_t>(t64);
            const uint32_t F = P ^ 1u;
            uint32_t nf = 0, nk = 0, kmin = kInf;
            for (uint32_t base = 0; base < st.np; base += 64) {
                const uint32_t i = base + lane;
                const bool valid = i < st.np;
                const uint32_t ic = valid ? i : 0u;
                const uint2 eb = L.lst[P][ic];
                const uint32_t e = eb.x;
                const uint32_t d = slot_dist(L, e & 0xFFFFu);
                const bool isF = valid && d < thr && d <= bound;
                const bool isK = valid && d >= thr && d <= bound;
                const bool drop = valid && d > bound;
                const uint64_t mF = __ballot(isF), mK = __ballot(isK);
                wave_sync();  // every lane has read its entry before the in-place compaction
                clear_pending(L, e & 0xFFFFu, drop);   // dropped: not pending
                *(isF ? &L.lst[F][nf + mbcnt(mF)] : L.sink()) = eb;
                *(isK ? &L.lst[P][nk + mbcnt(mK)] : L.sink()) = eb;
                kmin = min(kmin, isK ? d : kInf);
                nf += popc(mF);
                nk += popc(mK);
            }
            st.np = nk;
            st.tail = P * PC + nk;
            st.amask = 0xFFFFFFFFu;
            st.cap = PC;
            st.imin = kInf;
            wave_sync();
            for (uint32_t fb = 0; fb < nf && !st.ovf; fb += 64) {
                const uint32_t f = fb + lane;
                const bool valid = f < nf;
                const uint2 eb = L.lst[F][valid ? f : 0u];
                const uint32_t dd = slot_dist(L, valid ? (eb.x & 0xFFFFu) : lane);
                expand_chunk<HB, CT, 1>(L, st, c, a, &eb, &valid, &dd, bound);
            }
            if (st.ovf) break;
            pmin = min(wave_min(kmin), wave_min(st.imin));
        }
    }

    // ---- emit table entries in S, and clear the table for the next source
    bound = current_bound(c);
    uint2 *const stg = &L.lst[0][0];   // both lists, 2 PC entries: the search has ended
    uint32_t nst = 0, emitted = 0;
    unsigned long long warcs = 0;
    uint32_t wsettled = 0;
    for (uint32_t g0 = 0; g0 < static_cast<uint32_t>(H); g0 += 64 * U) {
        uint32_t k[U], d[U];
        bool occ[U], sb[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t slot = g0 + j * 64 + lane;
            occ[j] = read_slot(L, slot, c.voff, k[j], d[j]);
            sb[j] = !st.ovf && occ[j] && in_s(c, k[j]);
        }
        if (a.count_work && !st.ovf) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (occ[j] && d[j] <= bound) {
                    warcs += static_cast<unsigned long long>(a.row_ptr[c.rpo + k[j] + 1] - a.row_ptr[c.rpo + k[j]]);
                    wsettled += 1;
                }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) clear_slot(L, g0 + j * 64 + lane);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool m = sb[j] && d[j] <= bound;
            const uint64_t mM = __ballot(m);
            if (c.k && m) atomicAdd(&c.hist[kHistEmit + dist_bin(d[j])], 1u);
            emitted += popc(mM);
            *(m ? stg + nst + mbcnt(mM) : L.sink()) = make_uint2(d[j], k[j]);
            nst += popc(mM);
            if (nst + 64 > 2u * PC) {
                wave_sync();
                flush_pairs<HB, CT>(L, a, c, u, nst, stg);
            }
        }
    }
    wave_sync();
    flush_pairs<HB, CT>(L, a, c, u, nst, stg);
    if (c.k && emitted != 0) tighten_bound(c, tseen);
    if (a.count_work && !st.ovf) {
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(warcs & 0xFFFFFFFFull), o));
            const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(warcs >> 32), o));
            warcs += (static_cast<unsigned long long>(hi) << 32) | lo;
            wsettled += static_cast<uint32_t>(__shfl_xor(static_cast<int>(wsettled), o));
        }
        if (lane == 0) {
            atomicAdd(&a.ctl->arcs, warcs);
            atomicAdd(&a.ctl->settled, static_cast<unsigned long long>(wsettled));
        }
    }
    if (st.ovf && lane == 0) {
        const uint32_t idx = atomicAdd(a.novf, 1u);
        a.ovf[idx] = u;
        a.ovfq[idx] = c.q;
        if (a.first_tier) atomicAdd(&a.ctl->nretry, 1u);
    }
    wave_sync();
}

// The same search by a block of Tier<HB, CT>::NW waves sharing one table (tables
// of 2^12 entries and more, which leave room for few searches per CU):
// the ring of pending vertices is shared, each step the waves take 64
// vertices at most each (dealt round-robin), put back the ones far above the
// step's least distance (the deferral of the one-wave search) and expand the
// rest in windows of their own; appends reserve ring entries with LDS atomics.  Two block barriers
// per step; every loop that crosses a barrier decides on values read from
// LDS after a barrier, so the waves always agree.  The delta of the query
// is not used (one bucket, as with delta = 0: the distances are the same),
// nor the one-hop shortcut of k-closest pairs (the search finds those pairs).
template <int HB, bool CT>
__device__ void search_source_block(SearchLds<HB, CT> &L, BlockRing &B, const JoinArgs &a, const SrcCtx &c,
                                    int32_t u, unsigned long long &tseen) {
    constexpr int H = Tier<HB, CT>::H;
    constexpr int NW = Tier<HB, CT>::NW;
    constexpr int U = Tier<HB, CT>::U;
    constexpr uint32_t RC = 2u * Tier<HB, CT>::PC;
    const uint32_t lane = lane_id(), wv = wave_in_block();
    const int32_t ub = a.row_ptr[c.rpo + u];
    const int32_t ue = a.row_ptr[c.rpo + u + 1];
    uint2 *q = &L.lst[0][0];
    if (threadIdx.x == 0) {
        const uint32_t h0 = put_source(L, u, c.voff);   // the table is empty
        q[0] = make_uint2(h0 | (static_cast<uint32_t>(min(ue - ub, 0xFFFF)) << 16), static_cast<uint32_t>(ub));
        B.tail = 1;
        B.nins = 1;
        B.ovf = (ue - ub) > 0xFFFF ? 1u : 0u;
        B.dmin[0] = kInf;
        B.dmin[1] = kInf;
    }
    __syncthreads();
    WaveState st;
    st.np = 0;
    st.tail = 0;
    st.nins = 0;
    st.pnew = 0;
    st.imin = kInf;
    st.ovf = false;
    st.probing = false;
    st.amask = RC - 1u;
    st.cap = RC;
    st.blk = &B;
    uint32_t seen = 0, phase = 0, head = 0;
    while (true) {
        // after a barrier: every wave reads the same tail and overflow flag
        const uint32_t tail = B.tail;
        if (B.ovf != 0 || tail == head) break;
        if (c.hist != nullptr && phase >= 2) probe_phase(c, st.pnew, st.probing, seen);
        const uint32_t par = phase & 1u;
        ++phase;
        const uint32_t bound = current_bound(c);
        const uint32_t m = min(64u * NW, tail - head);
        // the step's entries dealt round-robin over the waves: with fewer
        // than 64 NW pending, every wave gets a share and no window is longer
        // than it needs to be
        const uint32_t mine = lane * NW + wv;
        bool valid = mine < m;
        const uint2 eb = q[(head + mine) & (RC - 1u)];
        const uint32_t es = valid ? (eb.x & 0xFFFFu) : lane;
        uint32_t dd = slot_dist(L, es);
        // taken entries stop being pending before the barrier: nothing is
        // relaxed between the last step's barrier and this one, so dd is the
        // distance the expansion uses, and a wave that improves one of these
        // vertices after the barrier finds it idle and queues it again
        clear_pending(L, es, valid);
        head += m;
        st.head = head;
        if (c.slack != kInf) {
            const uint32_t mn = wave_min(valid ? dd : kInf);
            if (lane == 0 && mn != kInf) atomicMin(&B.dmin[par], mn);
        }
        __syncthreads();   // every taken entry is read, the step's least distance complete
        if (threadIdx.x == 0) B.dmin[par ^ 1u] = kInf;   // for the next step (read after the next barrier)
        if (c.slack != kInf) {
            const uint32_t lim = sat_add(B.dmin[par], c.slack);
            bool later = valid && dd > lim && dd <= bound;
            if (__ballot(later) != 0) {
                // put back, pending again, unless a relaxation since the
                // barrier has queued the vertex already
                const bool queued = mark_pending(L, es, later);
                const bool app = later && !queued;
                const uint64_t mL = __ballot(app);
                uint32_t base = 0;
                if (lane == 0 && mL != 0) base = atomicAdd(&B.tail, popc(mL));
                base = readlane(base, 0);
                *(app ? q + ((base + mbcnt(mL)) & (RC - 1u)) : L.sink()) = eb;
            }
            valid = valid && !later;
        }
        expand_chunk<HB, CT, 1, false>(L, st, c, a, &eb, &valid, &dd, bound);
        __syncthreads();   // every append of the step is done
    }
    const bool ovf = B.ovf != 0;

    // ---- emit table entries in S (the waves take the table's chunks of 64 U
    // slots in turn, staged in each wave's slice of the ring, free once the
    // search has ended; the window areas take the sink writes), and clear the
    // table for the next source
    const uint32_t bound = current_bound(c);
    constexpr uint32_t SC = RC / NW;   // staging entries per wave
    static_assert(SC >= 128, "a wave's staging slice holds a flush threshold plus a chunk row");
    static_assert(H % (64 * U) == 0, "the table is a whole number of chunks");
    uint2 *stg = q + wv * SC;
    uint32_t nst = 0, emitted = 0;
    unsigned long long warcs = 0;
    uint32_t wsettled = 0;
    for (uint32_t g0 = wv * 64u * U; g0 < static_cast<uint32_t>(H); g0 += NW * 64u * U) {
        uint32_t k[U], d[U];
        bool occ[U], sb[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t slot = g0 + j * 64 + lane;
            occ[j] = read_slot(L, slot, c.voff, k[j], d[j]);
            sb[j] = !ovf && occ[j] && in_s(c, k[j]);
        }
        if (a.count_work && !ovf) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (occ[j] && d[j] <= bound) {
                    warcs += static_cast<unsigned long long>(a.row_ptr[c.rpo + k[j] + 1] - a.row_ptr[c.rpo + k[j]]);
                    wsettled += 1;
                }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) clear_slot(L, g0 + j * 64 + lane);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool mm = sb[j] && d[j] <= bound;
            const uint64_t mM = __ballot(mm);
            if (c.k && mm) atomicAdd(&c.hist[kHistEmit + dist_bin(d[j])], 1u);
            emitted += popc(mM);
            *(mm ? stg + nst + mbcnt(mM) : L.sink()) = make_uint2(d[j], k[j]);
            nst += popc(mM);
            if (nst + 64 > SC) {
                wave_sync();
                flush_pairs<HB, CT>(L, a, c, u, nst, stg);
            }
        }
    }
    wave_sync();
    flush_pairs<HB, CT>(L, a, c, u, nst, stg);
    if (c.k && emitted != 0) tighten_bound(c, tseen);
    if (a.count_work && !ovf) {
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(warcs & 0xFFFFFFFFull), o));
            const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(warcs >> 32), o));
            warcs += (static_cast<unsigned long long>(hi) << 32) | lo;
            wsettled += static_cast<uint32_t>(__shfl_xor(static_cast<int>(wsettled), o));
        }
        if (lane == 0) {
            atomicAdd(&a.ctl->arcs, warcs);
            atomicAdd(&a.ctl->settled, static_cast<unsigned long long>(wsettled));
        }
    }
    if (ovf && threadIdx.x == 0) {
        const uint32_t idx = atomicAdd(a.novf, 1u);
        a.ovf[idx] = u;
        a.ovfq[idx] = c.q;
        if (a.first_tier) atomicAdd(&a.ctl->nretry, 1u);
    }
    __syncthreads();   // the table is clear and B is free before the next source
}

__device__ __forceinline__ void launch_range(const JoinArgs &a, uint32_t &b, uint32_t &n) {
    b = a.sbeg ? *a.sbeg : 0u;
    const uint32_t e = *a.send;
    n = e > b ? e - b : 0u;
}

// One wavefront per block; the launch's sources split into 8 contiguous
// chunks, chunk c taken by the blocks with blockIdx % 8 == c so that each XCD
// (blocks are dealt to the 8 XCDs round-robin) sweeps one region of the
// source order and keeps its part of the graph in its own L2.  (Claiming
// sources through atomic counters instead was measured 1.6 times slower:
// thousands of blocks contend for the counters at a launch's start and end.)
// GEN = false: every source belongs to a theta-join, and the k-closest-pairs
// code is compiled out.
template <int HB, bool GEN, bool CT>
__global__ __launch_bounds__((64 * Tier<HB, CT>::NW)) void k_join(JoinArgs a) {
    __shared__ SearchLds<HB, CT> L;
    constexpr int H = Tier<HB, CT>::H;
    constexpr int NW = Tier<HB, CT>::NW;
    uint32_t b, n;
    launch_range(a, b, n);
    const uint32_t per = (n + 7u) / 8u;
    if (blockIdx.x >= 8u * per) return;
    // one k-query answered by k_kcp_direct: nothing to search
    if (GEN && a.srcq[b] == a.srcq[b + n - 1] && a.qs[a.srcq[b]].direct) return;
    for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(H); i += 64 * NW) clear_slot(L, i);
    if constexpr (NW > 1) {
        __shared__ BlockRing B;
        __syncthreads();
        unsigned long long tseen = 0;
        uint32_t tq = kInf;
        for (uint32_t t = blockIdx.x; t < 8u * per; t += gridDim.x) {
            const uint32_t si = (t & 7u) * per + (t >> 3);
            if (si >= n) continue;
            if (GEN && a.qs[a.srcq[b + si]].direct) continue;   // answered by k_kcp_direct
            SrcCtx c = load_ctx(a, a.srcq[b + si]);
            if (!GEN) {
                c.k = 0;
                c.hist = nullptr;
            }
            if (c.q != tq) {
                tq = c.q;
                tseen = 0;
            }
            search_source_block<HB, CT>(L, B, a, c, a.src[b + si], tseen);
        }
    } else {
        wave_sync();
        uint32_t tq = kInf;              // query of tseen
        unsigned long long tseen = 0;    // its emitted count at this wave's last bound update
        for (uint32_t t = blockIdx.x; t < 8u * per; t += gridDim.x) {
            const uint32_t si = (t & 7u) * per + (t >> 3);
            if (si >= n) continue;
            if (GEN && a.qs[a.srcq[b + si]].direct) continue;   // answered by k_kcp_direct
            SrcCtx c = load_ctx(a, a.srcq[b + si]);
            if (!GEN) {
                c.k = 0;
                c.hist = nullptr;
            }
            if (c.q != tq) {
                tq = c.q;
                tseen = 0;
            }
            if (GEN && c.k != 0 && !a.count_work &&
                static_cast<uint64_t>(current_bound(c)) < 2ull * static_cast<uint64_t>(c.wmin))
                direct_pairs<HB, CT>(L, a, c, a.src[b + si], tseen);
            else
                search_source<HB, CT>(L, a, c, a.src[b + si], tseen);
        }
    }
}

// ------------------------------------------------------------------ global-memory tier
// A search that outgrows every on-chip table runs here: one 1024-thread block
// per source, its distances in a dense per-slot array indexed by the local id.
// Distances are settled bucket by bucket (near-far delta-stepping with the
// query's gdelta): a round expands the near frontier (tentative distance below
// the bucket's end), improved vertices join the next near frontier or the far
// list; when no near vertex is left, the bucket end moves past the smallest
// far distance and the far list is split.  Without buckets, a frontier-
// synchronous search on a large road graph improves each vertex dozens of
// times; with them, close to once.
//
// A whole-graph search takes hundreds of rounds (about the graph's diameter
// in arcs), so a round's latency, not its work, sets the search's time, and
// the round is built to wait on global memory twice: for the arcs, then for
// one 64-bit atomicMin per arc.
//  - Each vertex has one word, (distance << 32) | 1 + the round of its last
//    improvement; round r's atomicMin with (nd << 32) | (r + 1) lowers the
//    distance only when nd is strictly smaller (an equal distance leaves the
//    word alone, since rounds only grow), and its old value tells whether the
//    vertex was already queued for round r + 1: improved in round r to a
//    distance below the bucket's end (an improvement in round r at or past the
//    end went to the far list instead, and a later one below it queues).
//  - The near frontier lives in LDS (kGF entries per round, the rest spills to
//    global memory) and carries each vertex's arc range, which the relaxed
//    arc's record holds, so no row pointer is read on the way.
//  - A frontier vertex's distance is read while its arcs load, the bound
//    (k-closest pairs) while the round's scan runs, and the S-bitmap word of
//    a relaxed arc's target (k-closest pairs, while discoveries are counted)
//    beside the atomic.  (One thread per frontier vertex relaxing its own arcs
//    instead of the flattened window was measured 1.4 times slower: a wave
//    whose vertices differ in degree repeats the arc-then-atomic chain.)
//  - Far-list membership needs no bitmap: every vertex with a finite distance
//    at or past the bucket's end is on the far list once, except vertices a
//    split dropped for lying beyond the bound (k-closest pairs: the bound
//    falls), whose word the split marks with round 0; so an improvement at or
//    past the bucket's end appends its vertex only if the vertex had no
//    distance or carries that mark.  Entries whose vertex later fell below the
//    bucket's end are dropped at the next split.
// An empty word is all ones (no distance, no round); rounds count from 1 per
// search and every word the search changed is reset at its end.
constexpr uint32_t kGT = 1024;
constexpr uint32_t kGJ = 4;                         // window arcs per lane
constexpr uint32_t kGWW = 64 * kGJ;                 // window arcs per wave
constexpr uint32_t kGF = 4096;                     // LDS frontier entries per round
constexpr unsigned long long kGEmpty = ~0ull;

// A slot's words are only touched by the block that owns the slot, so their
// loads and atomics are workgroup-scoped (served by the XCD's L2, which
// performs the atomics).
__device__ __forceinline__ unsigned long long gload64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned long long gmin64(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t word_dist(unsigned long long w) { return static_cast<uint32_t>(w >> 32); }

// Slot of a block-wide list append: one LDS atomic per wave.
__device__ __forceinline__ uint32_t block_append(bool want, uint32_t *counter) {
    const uint64_t m = __ballot(want);
    if (m == 0) return 0;
    const int leader = __ffsll(static_cast<long long>(m)) - 1;
    uint32_t base = 0;
    if (static_cast<int>(lane_id()) == leader) base = atomicAdd(counter, popc(m));
    return readlane(base, leader) + mbcnt(m);
}

// The LDS frontier of a global-tier search: two rounds' entries (vertex,
// first arc, arc count; by round parity), each wave's expansion window of
// kGWW arcs and the block's counters.  Frontier counts are kept by round
// modulo 3: round r reads count r, appends to count r + 1 and clears count
// r + 2 (round r - 1's, read by then), so that no barrier inside a round is
// needed before its appends.
struct GlobalLds {
    uint32_t fy[2][kGF];
    int32_t fb[2][kGF];
    uint32_t fd[2][kGF];
    int32_t widx[kGT / 64][kGWW];    // per wave: window arc index
    uint8_t worig[kGT / 64][kGWW];   //   and the lane whose vertex it leaves
    uint32_t nf[3];                  // frontier entries, by round modulo 3
    uint32_t ntouched, bound, probing, nfar, kept, dmin, dnext;
};

// Append vertex y (global id; arcs [beg, beg + deg)) to the frontier of
// parity p (count ci) when want: LDS entries first, then the spill array.
__device__ __forceinline__ void frontier_push(GlobalLds &G, uint32_t p, uint32_t ci, uint32_t *spill, bool want,
                                              uint32_t y, int32_t beg, uint32_t deg) {
    const uint32_t i = block_append(want, &G.nf[ci]);
    if (!want) return;
    if (i < kGF) {
        G.fy[p][i] = y;
        G.fb[p][i] = beg;
        G.fd[p][i] = deg;
    } else {
        spill[i - kGF] = y;
    }
}

__global__ __launch_bounds__(1024) void k_join_global(JoinArgs a, uint32_t *slots, uint32_t nslots,
                                                      int32_t Vmax) {
    __shared__ GlobalLds G;
    __shared__ uint32_t s_si;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    uint32_t sb, n;
    launch_range(a, sb, n);
    const size_t V = static_cast<size_t>(Vmax), NV = nslots * V;
    const size_t k = blockIdx.x;
    unsigned long long *word = reinterpret_cast<unsigned long long *>(slots) + k * V;   // local ids
    uint32_t *spill0 = slots + 2 * NV + k * V;                      // global ids
    uint32_t *spill1 = spill0 + NV;
    uint32_t *touched = spill1 + NV;                                // local ids
    uint32_t *far = touched + NV;                                   // local ids
    // sources: block b takes source b, then claims the next unclaimed one
    // through the launch's counter (whole-graph searches differ widely in
    // length, and the grid holds at most one block per slot)
    for (uint32_t i = blockIdx.x; i < n;) {
        const int32_t u = a.src[sb + i];
        const SrcCtx c = load_ctx(a, a.srcq[sb + i]);
        const uint32_t voff = static_cast<uint32_t>(c.voff);
        // a k-query answered by k_kcp_direct has nothing to search
        if (c.k != 0 && a.qs[c.q].direct) {
            __syncthreads();   // every thread has read the query before the claim is rewritten
            if (tid == 0) s_si = gridDim.x + atomicAdd(a.work, 1u);
            __syncthreads();
            i = s_si;
            continue;
        }
        if (tid == 0) {
            word[u - c.voff] = 1ull;   // distance 0, queued for round 1
            G.fy[1][0] = static_cast<uint32_t>(u);
            G.fb[1][0] = a.row_ptr[c.rpo + u];
            G.fd[1][0] = static_cast<uint32_t>(a.row_ptr[c.rpo + u + 1] - G.fb[1][0]);
            touched[0] = static_cast<uint32_t>(u - c.voff);
            G.nf[1] = 1;   // round 1
            G.nf[2] = 0;
            G.nf[0] = 0;
            G.probing = 0;
            G.ntouched = 1;
            G.nfar = 0;
            G.bound = current_bound(c);
        }
        __syncthreads();
        uint32_t seen = 0, pnew = 0, round = 1;
        const uint32_t gdelta = a.qd[c.q].gdelta;
        uint32_t thr = gdelta;   // end of the current bucket (exclusive)
        bool probing = false;
        while (true) {
            const uint32_t cur = round & 1u, nxt = cur ^ 1u;
            const uint32_t cf = round % 3u, af = (round + 1u) % 3u, zf = (round + 2u) % 3u;
            uint32_t *spill_cur = cur ? spill1 : spill0, *spill_nxt = cur ? spill0 : spill1;
            if (G.nf[cf] == 0) {
                // no near vertex left: everything below thr is settled
                const uint32_t nfar = G.nfar;
                if (nfar == 0) break;
                if (tid == 0) {
                    G.dmin = kInf;
                    G.kept = 0;
                    G.bound = current_bound(c);
                }
                __syncthreads();
                const uint32_t bound = G.bound;
                uint32_t dmin = kInf;
                for (uint32_t j = tid; j < nfar; j += kGT) {
                    const uint32_t d = word_dist(gload64(&word[far[j]]));
                    if (d >= thr && d <= bound) dmin = min(dmin, d);
                }
                dmin = wave_min(dmin);
                if (lane == 0 && dmin != kInf) atomicMin(&G.dmin, dmin);
                __syncthreads();
                const uint32_t told = thr;
                if (G.dmin != kInf) {
                    const uint64_t t = (static_cast<uint64_t>(G.dmin) / gdelta + 1ull) * gdelta;
                    thr = t > kInf ? kInf : static_cast<uint32_t>(t);
                }
                // split the far list in place: settled or out of bound -> dropped,
                // inside the new bucket -> near frontier, beyond it -> kept
                for (uint32_t cb = 0; cb < nfar; cb += kGT) {
                    const uint32_t j = cb + tid;
                    const bool valid = j < nfar;
                    const uint32_t yl = valid ? far[j] : 0u;
                    const uint32_t d = valid ? word_dist(gload64(&word[yl])) : kInf;
                    __syncthreads();   // the chunk is read before kept entries overwrite it
                    const bool near = valid && d >= told && d < thr && d <= bound;
                    const bool keep = valid && d >= thr && d <= bound;
                    if (valid && d != kInf && d > bound)   // dropped: marked, so that it can join again
                        word[yl] = static_cast<unsigned long long>(d) << 32;
                    const uint32_t y = yl + voff;
                    const int32_t beg = near ? a.row_ptr[c.rpo + y] : 0;
                    const uint32_t deg = near ? static_cast<uint32_t>(a.row_ptr[c.rpo + y + 1] - beg) : 0u;
                    frontier_push(G, cur, cf, spill_cur, near, y, beg, deg);
                    const uint32_t ki = block_append(keep, &G.kept);
                    if (keep) far[ki] = yl;
                    __syncthreads();
                }
                if (tid == 0) G.nfar = G.kept;
                __syncthreads();
                continue;
            }
            const uint32_t nf = G.nf[cf];
            if (tid == 0) G.nf[zf] = 0;   // (read in round - 1; appended to from round + 1 on)
            // each wave expands 64 frontier entries at a time with a window of
            // its own: no block barrier until the round's end
            const uint32_t bound = current_bound(c);
            const bool probe_on = G.probing != 0;
            const uint32_t wv = tid >> 6;
            for (uint32_t cb = wv * 64u; cb < nf; cb += kGT) {
                const uint32_t t = cb + lane;
                const bool valid = t < nf;
                uint32_t y = 0, deg = 0;
                int32_t beg = 0;
                if (valid) {
                    if (t < kGF) {
                        y = G.fy[cur][t];
                        beg = G.fb[cur][t];
                        deg = G.fd[cur][t];
                    } else {
                        y = spill_cur[t - kGF];
                        beg = a.row_ptr[c.rpo + y];
                        deg = static_cast<uint32_t>(a.row_ptr[c.rpo + y + 1] - beg);
                    }
                }
                // the vertex's current distance, read while the scan and the arcs
                // proceed (an entry queued earlier may have improved since)
                const uint32_t dl = valid ? word_dist(gload64(&word[y - voff])) : kInf;
                const uint32_t incl = wave_incl_scan(deg);
                const uint32_t excl = incl - deg;
                const uint32_t total = readlane(incl, 63);
                for (uint32_t wb = 0; wb < total; wb += kGWW) {
                    const uint32_t lo = max(excl, wb), hi = min(excl + deg, wb + kGWW);
                    for (uint32_t p = lo; p < hi; ++p) {
                        G.widx[wv][p - wb] = beg + static_cast<int32_t>(p - excl);
                        G.worig[wv][p - wb] = static_cast<uint8_t>(lane);
                    }
                    const uint32_t cnt = min(kGWW, total - wb);
                    ArcRec r[kGJ];
                    uint32_t org[kGJ];
#pragma unroll
                    for (uint32_t j = 0; j < kGJ; ++j) {
                        const uint32_t e = j * 64u + lane;
                        r[j] = a.arcs[e < cnt ? G.widx[wv][e] : 0];
                        org[j] = e < cnt ? G.worig[wv][e] : 64u;
                    }
                    wave_sync();   // the window map is read before the next window rewrites it
                    uint32_t nd[kGJ];
#pragma unroll
                    for (uint32_t j = 0; j < kGJ; ++j) {
                        // the tail's distance, from the lane expanding it
                        const uint32_t od = static_cast<uint32_t>(
                            __builtin_amdgcn_ds_bpermute(static_cast<int>((org[j] & 63u) << 2), static_cast<int>(dl)));
                        nd[j] = org[j] < 64u ? sat_add(od, r[j].w) : kInf;
                    }
                    unsigned long long old[kGJ];
                    uint32_t sw[kGJ];   // (k-closest pairs, counting: the S-bitmap word of the target)
#pragma unroll
                    for (uint32_t j = 0; j < kGJ; ++j) {
                        // (nd < kInf: a word is changed only with a real distance,
                        // so every changed word is on the touched list)
                        const uint32_t yl = static_cast<uint32_t>(r[j].y) - voff;
                        const bool go = nd[j] <= bound && nd[j] < kInf;
                        old[j] = go ? gmin64(&word[yl], (static_cast<unsigned long long>(nd[j]) << 32) | (round + 1u)) : 0ull;
                        // read beside the atomic rather than after it
                        sw[j] = (go && probe_on) ? c.sbits[yl >> 5] : 0u;
                    }
                    // what each relaxation appends: its vertex to the touched list
                    // (first distance), the next round's frontier (below the
                    // bucket's end, not queued yet) or the far list; the wave's
                    // places on the three lists come from one LDS atomic each, issued
                    // together
                    uint64_t mt[kGJ], mq[kGJ], mf[kGJ];
                    uint32_t nt = 0, nq = 0, nfr = 0;
#pragma unroll
                    for (uint32_t j = 0; j < kGJ; ++j) {
                        const uint32_t od = word_dist(old[j]);
                        const bool imp = nd[j] < od;
                        const bool queued = static_cast<uint32_t>(old[j]) == round + 1u && od < thr;
                        mt[j] = __ballot(imp && od == kInf);
                        mq[j] = __ballot(imp && nd[j] < thr && !queued);
                        mf[j] = __ballot(imp && nd[j] >= thr && (od == kInf || static_cast<uint32_t>(old[j]) == 0u));
                        nt += popc(mt[j]);
                        nq += popc(mq[j]);
                        nfr += popc(mf[j]);
                    }
                    uint32_t bt = 0, bq = 0, bf = 0;
                    if (lane == 0) {
                        if (nt) bt = atomicAdd(&G.ntouched, nt);
                        if (nq) bq = atomicAdd(&G.nf[af], nq);
                        if (nfr) bf = atomicAdd(&G.nfar, nfr);
                    }
                    bt = readlane(bt, 0);
                    bq = readlane(bq, 0);
                    bf = readlane(bf, 0);
#pragma unroll
                    for (uint32_t j = 0; j < kGJ; ++j) {
                        const uint32_t yl = static_cast<uint32_t>(r[j].y) - voff;
                        const uint64_t bit = 1ull << lane;
                        if (mt[j] & bit) {
                            touched[bt + mbcnt(mt[j])] = yl;
                            if ((sw[j] >> (yl & 31u)) & 1u) {
                                atomicAdd(&probe_hist(c)[dist_bin(nd[j])], 1u);
                                atomicAdd(probe_count(c), 1u);
                            }
                        }
                        if (mq[j] & bit) {
                            const uint32_t fi = bq + mbcnt(mq[j]);
                            if (fi < kGF) {
                                G.fy[nxt][fi] = static_cast<uint32_t>(r[j].y);
                                G.fb[nxt][fi] = r[j].ybeg;
                                G.fd[nxt][fi] = static_cast<uint32_t>(r[j].yend - r[j].ybeg);
                            } else {
                                spill_nxt[fi - kGF] = static_cast<uint32_t>(r[j].y);
                            }
                        }
                        if (mf[j] & bit) far[bf + mbcnt(mf[j])] = yl;
                        bt += popc(mt[j]);
                        bq += popc(mq[j]);
                        bf += popc(mf[j]);
                    }
                }
            }
            // (k-closest pairs, every 8th round, wave 0) the discovery count
            // lowers the bound; whether to keep counting is read next round
            if (tid < 64 && c.hist != nullptr && (round & 7u) == 1u) {
                probe_phase(c, pnew, probing, seen);
                if (tid == 0) G.probing = probing ? 1u : 0u;
            }
            ++round;
            __syncthreads();
        }
        // emit S members, count work, reset the slot
        if (tid == 0) G.bound = current_bound(c);
        __syncthreads();
        const uint32_t bound = G.bound;
        const uint32_t nt = G.ntouched;
        unsigned long long warcs = 0;
        uint32_t wsettled = 0;
        for (uint32_t j0 = 0; j0 < nt; j0 += kGT) {
            const uint32_t j = j0 + tid;
            uint32_t yl = 0, d = kInf;
            bool m = false;
            if (j < nt) {
                yl = touched[j];
                d = word_dist(gload64(&word[yl]));
                word[yl] = kGEmpty;
                m = d <= bound && ((c.sbits[yl >> 5] >> (yl & 31u)) & 1u);
                if (a.count_work && d <= bound) {
                    warcs += static_cast<unsigned long long>(a.row_ptr[c.rpo + yl + voff + 1] -
                                                             a.row_ptr[c.rpo + yl + voff]);
                    wsettled += 1;
                }
            }
            const uint64_t mm = __ballot(m);
            if (c.k && m) atomicAdd(&c.hist[kHistEmit + dist_bin(d)], 1u);
            if (mm != 0) {
                unsigned long long base = 0;
                if (lane == 0) {
                    base = atomicAdd(&a.ctl->npairs, static_cast<unsigned long long>(popc(mm)));
                    atomicAdd(&c.qs->npairs, static_cast<unsigned long long>(popc(mm)));
                }
                const uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(base & 0xFFFFFFFFull), 0));
                const uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(base >> 32), 0));
                base = (static_cast<unsigned long long>(hi) << 32) | lo;
                const unsigned long long idx = base + mbcnt(mm);
                if (m && idx < a.rec_cap) {
                    Rec rr;
                    const int32_t cy = caller_id(a, static_cast<int32_t>(yl) + c.voff, c.voff);
                    const int32_t cu = caller_id(a, u, c.voff);
                    rr.u = c.swapped ? cy : cu;
                    rr.v = c.swapped ? cu : cy;
                    rr.d = d;
                    rr.q = c.q;
                    if (a.bins) rr.q |= bin_place(atomicAdd(&a.bins[a.binbase[c.q] + d], 1u));
                    a.recs[idx] = rr;
                }
            }
        }
        if (a.count_work) {
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(warcs & 0xFFFFFFFFull), o));
                const uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(warcs >> 32), o));
                warcs += (static_cast<unsigned long long>(hi) << 32) | lo;
                wsettled += static_cast<uint32_t>(__shfl_xor(static_cast<int>(wsettled), o));
            }
            if (lane == 0) {
                atomicAdd(&a.ctl->arcs, warcs);
                atomicAdd(&a.ctl->settled, static_cast<unsigned long long>(wsettled));
            }
        }
        __syncthreads();
        unsigned long long tseen = 0;
        if (c.k && tid < 64) tighten_bound(c, tseen);
        if (tid == 0) s_si = gridDim.x + atomicAdd(a.work, 1u);
        __syncthreads();   // the slot is clean before the next source starts
        i = s_si;
        __syncthreads();   // every thread has the claim before the next one is written
    }
}

// ------------------------------------------------------------------ staging
__global__ __launch_bounds__(256) void k_publish(const uint32_t *src, uint32_t *dst, uint32_t words) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < words) dst[i] = src[i];
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Largest p in [0, n) with a[p] <= x (a non-decreasing, a[0] <= x).
template <typename T>
__device__ __forceinline__ uint32_t seg_of(const T *a, uint32_t n, T x) {
    uint32_t lo = 0, hi = n;   // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// One thread per element of the flattened (S then R) lists of every query in
// staging order: range and duplicate checks, S bits, and rank bits of R.
__global__ void k_mark(CallBuffers b, const int32_t *rank) {
    const unsigned long long i = blockIdx.x * static_cast<unsigned long long>(blockDim.x) + threadIdx.x;
    const uint32_t nq = static_cast<uint32_t>(b.nq);
    if (i >= b.ebase[nq]) return;
    const uint32_t p = seg_of(b.ebase, nq, i);
    const uint32_t q = b.perm[p];
    const QueryDesc &d = b.qd[q];
    const unsigned long long j = i - b.ebase[p];
    uint32_t err = 0;
    if (j < static_cast<unsigned long long>(d.nS)) {
        const int32_t s0 = d.S[j];
        if (s0 < 0 || s0 >= d.V) {
            err = kErrRange;
        } else {
            const int32_t s = rank ? rank[d.voff + s0] : s0;   // local id in the device copy
            const uint32_t bit = 1u << (s & 31);
            if (atomicOr(&b.sbits[d.sbits + (s >> 5)], bit) & bit) err = kErrDupS;
        }
    } else {
        const int32_t u = d.R[j - d.nS];
        if (u < 0 || u >= d.V) {
            err = kErrRange;
        } else {
            const int32_t r = rank ? rank[d.voff + u] : u;
            const uint32_t bit = 1u << (r & 31);
            if (atomicOr(&b.rbits[d.rbits + (r >> 5)], bit) & bit) err = kErrDupR;
        }
    }
    if (err) {
        atomicOr(&b.qs[q].err, err);
        atomicOr(&b.ctl->err, err);
    }
}

// R and S must be disjoint: element i of the flattened lists, if it is in
// some R, must not be in that query's S.
__device__ __forceinline__ void check_overlap(const CallBuffers &b, const int32_t *rank, unsigned long long i) {
    const uint32_t nq = static_cast<uint32_t>(b.nq);
    if (i >= b.ebase[nq]) return;
    const uint32_t p = seg_of(b.ebase, nq, i);
    const uint32_t q = b.perm[p];
    const QueryDesc &d = b.qd[q];
    const unsigned long long j = i - b.ebase[p];
    if (j < static_cast<unsigned long long>(d.nS)) return;
    const int32_t u0 = d.R[j - d.nS];
    if (u0 < 0 || u0 >= d.V) return;
    const int32_t u = rank ? rank[d.voff + u0] : u0;   // local id in the device copy
    if ((b.sbits[d.sbits + (u >> 5)] >> (u & 31)) & 1u) {
        atomicOr(&b.qs[q].err, kErrOverlap);
        atomicOr(&b.ctl->err, kErrOverlap);
    }
}

// Block-wide exclusive scan of one value per thread (blockDim.x = 1024); *total
// receives the block sum.  Uses wsum[16] in LDS.
__device__ __forceinline__ uint32_t block_excl_scan_1024(uint32_t v, uint32_t *wsum, uint32_t *total) {
    const uint32_t tid = threadIdx.x;
    const uint32_t incl = wave_incl_scan(v);
    if ((tid & 63u) == 63u) wsum[tid >> 6] = incl;
    __syncthreads();
    uint32_t off = 0, all = 0;
    for (uint32_t w = 0; w < 16; ++w) {
        const uint32_t x = wsum[w];
        off += w < (tid >> 6) ? x : 0u;
        all += x;
    }
    __syncthreads();
    *total = all;
    return off + incl - v;
}

// After the marks, in one launch: the disjointness check (thread i takes
// element i of the flattened lists) and source listing pass 1, the marked
// ranks per 1024-word block of the rank pool (the first nblk blocks).
__global__ __launch_bounds__(1024) void k_overlap_count(CallBuffers b, const int32_t *rank, uint32_t nblk) {
    __shared__ uint32_t wsum[16];
    check_overlap(b, rank, blockIdx.x * 1024ull + threadIdx.x);
    if (blockIdx.x >= nblk) return;
    const uint32_t i = blockIdx.x * 1024u + threadIdx.x;
    uint32_t total;
    block_excl_scan_1024(i < b.rwords ? __popc(b.rbits[i]) : 0u, wsum, &total);
    if (threadIdx.x == 0) b.stage_scratch[blockIdx.x] = total;
}

// Source listing, pass 2: list the marked ranks in increasing pool order as
// global vertex ids with their queries; the first word of each query records
// where its sources start.
__global__ __launch_bounds__(1024) void k_rank_emit(CallBuffers b, const uint32_t *bsum) {
    __shared__ uint32_t wsum[16];
    const uint32_t tid = threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t j = tid; j < blockIdx.x; j += 1024) acc += bsum[j];
    uint32_t pre;
    block_excl_scan_1024(acc, wsum, &pre);
    const uint32_t i = blockIdx.x * 1024u + tid;
    const bool valid = i < b.rwords;
    uint32_t bits = valid ? b.rbits[i] : 0u;
    uint32_t total;
    uint32_t pos = pre + block_excl_scan_1024(__popc(bits), wsum, &total);
    if (valid) {
        const uint32_t p = seg_of(b.rbase, static_cast<uint32_t>(b.nq), i);
        const uint32_t q = b.perm[p];
        const uint32_t lw = i - b.rbase[p];
        const int32_t voff = b.qd[q].voff;
        if (lw == 0) b.qs[q].src_start = pos;
        while (bits) {
            const uint32_t bt = __ffs(bits) - 1u;
            const int32_t r = static_cast<int32_t>(lw * 32u + bt);
            b.src[pos] = voff + r;   // the rank is the local id in the device copy
            b.srcq[pos] = q;
            ++pos;
            bits &= bits - 1u;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) b.ctl->nsrc = pre + total;
}

// ------------------------------------------------------------------ k-closest pairs
// Seed: every distinct (u, y) with u in R, y in S joined by an arc has
// dist(u, y) <= the lightest such arc's weight, so the bin edge where k of
// these weights are reached bounds the k-th smallest distance.  A pair with
// parallel arcs is counted once, at its first lightest arc.
__global__ __launch_bounds__(256) void k_kcp_seed_hist(JoinArgs a) {
    __shared__ uint32_t h[kDistBins];
    const uint32_t n = *a.send;
    const uint32_t first = blockIdx.x * blockDim.x;
    if (first >= n) return;
    const uint32_t i = first + threadIdx.x;
    // sources are listed query by query, so the block's sources belong to one
    // query when its first and last do: then count in LDS, one global atomic per bin
    const uint32_t last = min(first + blockDim.x, n) - 1u;
    const bool one = a.srcq[first] == a.srcq[last];
    if (one) {
        for (uint32_t j = threadIdx.x; j < kDistBins; j += blockDim.x) h[j] = 0;
        __syncthreads();
    }
    if (i < n) {
        const SrcCtx c = load_ctx(a, a.srcq[i]);
        if (c.k != 0) {
            uint32_t *seed = c.hist + kHistSeed;
            const int32_t u = a.src[i];
            const int32_t b = a.row_ptr[c.rpo + u], e = a.row_ptr[c.rpo + u + 1];
            for (int32_t x = b; x < e; ++x) {
                const ArcRec r = a.arcs[x];
                if (!first_of_pair(a, x) || !in_s(c, static_cast<uint32_t>(r.y))) continue;
                atomicAdd(one ? &h[dist_bin(r.w)] : &seed[dist_bin(r.w)], 1u);
            }
        }
    }
    if (one) {
        __syncthreads();
        const SrcCtx c = load_ctx(a, a.srcq[first]);
        if (c.k != 0)
            for (uint32_t j = threadIdx.x; j < kDistBins; j += blockDim.x)
                if (h[j]) atomicAdd(&c.hist[kHistSeed + j], h[j]);
    }
}

// One wave per query: the seeded bound of each k-query, capped by its theta,
// and whether every pair within it is a direct arc (allow_direct: not when
// the searches count their work).
__global__ __launch_bounds__(64) void k_kcp_seed_bound(const QueryDesc *qd, QueryState *qs, const uint32_t *hists,
                                                       int allow_direct) {
    const QueryDesc &d = qd[blockIdx.x];
    if (d.k == 0) return;
    const uint32_t b = min(wave_bound_from_hist(hists + d.hist + kHistSeed, d.k), d.theta);
    if (threadIdx.x == 0) {
        qs[blockIdx.x].bound = b;
        qs[blockIdx.x].direct =
            allow_direct && static_cast<uint64_t>(b) < 2ull * static_cast<uint64_t>(d.wmin) ? 1u : 0u;
    }
}

// k-closest pairs whose seeded bound is below twice the lightest arc: every
// path of two or more arcs is longer, so the pairs within the bound are the
// direct arcs from a source into S no heavier than it, each at the weight of
// the pair's lightest arc (parallel arcs: the first lightest).  One thread
// per source (a source has a few arcs, so a wave per source would idle): its
// arcs are read kDirectBatch at a time with every load of a batch issued
// before any is used, the records of a wave's sources of one query are
// reserved with one pair of atomics, then written.  The query's searches are
// skipped.
constexpr int kDirectBatch = 8;

// Bit k: arc x0 + k (below e) gives a pair.  Arcs past e read arc x0 (x0 < e)
// and fail.
__device__ __forceinline__ uint32_t direct_batch(const JoinArgs &a, const SrcCtx &c, int32_t x0, int32_t e,
                                                 uint32_t bound, ArcRec *r) {
    uint32_t fb[kDirectBatch], sb[kDirectBatch];
#pragma unroll
    for (int k = 0; k < kDirectBatch; ++k) r[k] = a.arcs[x0 + k < e ? x0 + k : x0];
#pragma unroll
    for (int k = 0; k < kDirectBatch; ++k) {
        const int32_t x = x0 + k < e ? x0 + k : x0;
        const uint32_t yl = static_cast<uint32_t>(r[k].y) - static_cast<uint32_t>(c.voff);
        fb[k] = a.first[static_cast<uint32_t>(x) >> 5] >> (x & 31);
        sb[k] = c.sbits[yl >> 5] >> (yl & 31u);
    }
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < kDirectBatch; ++k)
        m |= (x0 + k < e && r[k].w <= bound && (fb[k] & sb[k] & 1u) != 0u) ? (1u << k) : 0u;
    return m;
}

__global__ __launch_bounds__(256) void k_kcp_direct(JoinArgs a) {
    const uint32_t n = *a.send;
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    const uint32_t lane = lane_id();
    uint32_t q = 0;
    bool act = false;
    if (i < n) {
        q = a.srcq[i];
        act = a.qs[q].direct != 0;
    }
    const uint64_t mact = __ballot(act);
    if (mact == 0) return;   // wave-uniform
    SrcCtx c{};
    uint32_t bound = 0, cnt = 0, m0 = 0;
    int32_t u = 0, b = 0, e = 0;
    ArcRec r[kDirectBatch];
    if (act) {
        c = load_ctx(a, q);
        bound = c.qs->bound;
        u = a.src[i];
        b = a.row_ptr[c.rpo + u];
        e = a.row_ptr[c.rpo + u + 1];
        m0 = b < e ? direct_batch(a, c, b, e, bound, r) : 0u;   // (a batch reads arc x0 < e)
        cnt = popc(m0);
        for (int32_t x0 = b + kDirectBatch; x0 < e; x0 += kDirectBatch) {   // sources of many arcs
            ArcRec t[kDirectBatch];
            cnt += popc(direct_batch(a, c, x0, e, bound, t));
        }
    }
    // reserve: the lanes of the first active lane's query together, the rest alone
    const int first = __ffsll(static_cast<unsigned long long>(mact)) - 1;
    const uint32_t q0 = static_cast<uint32_t>(__shfl(static_cast<int>(q), first));
    const bool same = act && q == q0;
    const uint32_t cs = same ? cnt : 0u;
    const uint32_t incl = wave_incl_scan(cs);
    const uint32_t tot = readlane(incl, 63);
    unsigned long long base = 0;
    if (tot != 0) {
        uint32_t lo = 0, hi = 0;
        if (static_cast<int>(lane) == first) {
            const unsigned long long w = atomicAdd(&a.ctl->npairs, static_cast<unsigned long long>(tot));
            atomicAdd(&a.qs[q0].npairs, static_cast<unsigned long long>(tot));
            lo = static_cast<uint32_t>(w);
            hi = static_cast<uint32_t>(w >> 32);
        }
        base = (static_cast<unsigned long long>(static_cast<uint32_t>(__shfl(static_cast<int>(hi), first))) << 32) |
               static_cast<uint32_t>(__shfl(static_cast<int>(lo), first));
        base += incl - cs;
    }
    if (act && !same && cnt != 0) {
        base = atomicAdd(&a.ctl->npairs, static_cast<unsigned long long>(cnt));
        atomicAdd(&c.qs->npairs, static_cast<unsigned long long>(cnt));
    }
    if (!act || cnt == 0) return;
    unsigned long long idx = base;
    const int32_t from = caller_id(a, u, c.voff);
    for (int32_t x0 = b; x0 < e; x0 += kDirectBatch) {
        uint32_t m = m0;
        if (x0 != b) m = direct_batch(a, c, x0, e, bound, r);
#pragma unroll
        for (int k = 0; k < kDirectBatch; ++k) {
            if (!((m >> k) & 1u)) continue;
            atomicAdd(&c.hist[kHistEmit + dist_bin(r[k].w)], 1u);
            if (idx < a.rec_cap) {
                const int32_t to = caller_id(a, r[k].y, c.voff);
                Rec o;
                o.u = c.swapped ? to : from;
                o.v = c.swapped ? from : to;
                o.d = r[k].w;
                o.q = q;
                a.recs[idx] = o;
            }
            ++idx;
        }
    }
}

// Keep the records within their query's final bound (order is restored by the
// sort).  Each block takes a contiguous tile: it counts the records it keeps,
// reserves their places with one global atomic, then writes them; only
// k-closest-pairs queries count their kept records (every record of a
// theta-join is kept, so its count is its emitted count).
__device__ __forceinline__ bool keep_rec(const CallBuffers &b, const Rec &r) {
    return b.qd[r.q].k == 0 || r.d <= b.qs[r.q].bound;
}

__global__ __launch_bounds__(256) void k_select(CallBuffers b) {
    __shared__ uint32_t s_cnt;
    __shared__ unsigned long long s_base;
    const unsigned long long n = min(b.ctl->npairs, b.rec_cap);
    const Rec *in = b.recs[0];
    Rec *kept = b.recs[1];
    const unsigned long long per = ((n + gridDim.x - 1) / gridDim.x + 255ull) / 256ull * 256ull;
    const unsigned long long beg = min(n, blockIdx.x * per), end = min(n, beg + per);
    if (beg >= end) return;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    uint32_t mine = 0;
    for (unsigned long long i0 = beg; i0 < end; i0 += 256) {
        const unsigned long long i = i0 + threadIdx.x;
        bool kq = false;
        uint32_t q = 0;
        if (i < end) {
            const Rec r = in[i];
            const bool keep = keep_rec(b, r);
            mine += keep ? 1u : 0u;
            q = r.q;
            kq = keep && b.qd[r.q].k != 0;
        }
        // the query's kept count: one atomic per query and wave (lanes find the
        // lanes of their query by its 16 bits; a call's records mostly share
        // a few queries, and per-record atomics on one word serialise)
        uint64_t peers = __ballot(kq);
        if (peers != 0) {
#pragma unroll
            for (int bit = 0; bit < 16; ++bit) {
                const bool set = (q >> bit) & 1u;
                const uint64_t m = __ballot(kq && set);
                peers &= set ? m : ~m;
            }
            if (kq && mbcnt(peers) == 0) atomicAdd(&b.qs[q].nsel, static_cast<unsigned long long>(popc(peers)));
        }
    }
    for (int o = 32; o > 0; o >>= 1) mine += static_cast<uint32_t>(__shfl_xor(static_cast<int>(mine), o));
    if (lane_id() == 0 && mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        s_base = s_cnt ? atomicAdd(&b.ctl->nsel, static_cast<unsigned long long>(s_cnt)) : 0ull;
        s_cnt = 0;
    }
    __syncthreads();
    for (unsigned long long i0 = beg; i0 < end; i0 += 256) {
        const unsigned long long i = i0 + threadIdx.x;
        Rec r{0, 0, 0, 0};
        bool keep = false;
        if (i < end) {
            r = in[i];
            keep = keep_rec(b, r);
        }
        const uint64_t mk = __ballot(keep);
        if (mk == 0) continue;
        uint32_t base = 0;
        if (lane_id() == 0) base = atomicAdd(&s_cnt, popc(mk));
        base = readlane(base, 0);
        if (keep) kept[s_base + base + mbcnt(mk)] = r;
    }
}

// ------------------------------------------------------------------ layout
// Exclusive scan of 64-bit values over a 1024-thread block: a shuffle scan
// within each wave, then each thread adds the totals of the waves before it
// (s: at least 16 words; two block barriers).
__device__ __forceinline__ unsigned long long block_excl_scan_u64(unsigned long long v, unsigned long long *s,
                                                                  unsigned long long *total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    unsigned long long incl = v;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const unsigned long long x = __shfl_up(incl, o, 64);
        incl += lane >= o ? x : 0ull;
    }
    if (lane == 63u) s[w] = incl;
    __syncthreads();
    unsigned long long off = 0, all = 0;
    for (uint32_t i = 0; i < 16; ++i) {
        const unsigned long long x = s[i];
        off += i < w ? x : 0ull;
        all += x;
    }
    __syncthreads();
    *total = all;
    return off + incl - v;
}

__device__ __forceinline__ uint32_t bitlen32(uint32_t x) { return x ? 32u - static_cast<uint32_t>(__clz(x)) : 0u; }

// One block: per query the kept count, its first position in the sorted
// order, its output count (0 for a query with an argument error) and output
// offset; then the sort key layout from the largest kept distance bound.
__device__ __forceinline__ void layout_block(const CallBuffers &b, int selected, uint32_t qb, uint32_t vb,
                                             unsigned long long *s, uint32_t &s_dmax) {
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_dmax = 0;
    __syncthreads();   // cleared before any thread raises it
    unsigned long long cs = 0, co = 0;
    for (uint32_t q0 = 0; q0 < static_cast<uint32_t>(b.nq); q0 += 1024) {
        const uint32_t q = q0 + tid;
        const bool valid = q < static_cast<uint32_t>(b.nq);
        unsigned long long nsel = 0, nout = 0;
        if (valid) {
            const QueryDesc &d = b.qd[q];
            const QueryState &st = b.qs[q];
            nsel = (selected && d.k) ? st.nsel : st.npairs;   // a theta-join keeps every record
            nout = st.err ? 0ull : (d.k ? min(nsel, static_cast<unsigned long long>(d.k)) : nsel);
            if (nsel) atomicMax(&s_dmax, d.k ? st.bound : d.theta);
        }
        unsigned long long ts, to;
        const unsigned long long es = block_excl_scan_u64(nsel, s, &ts);
        const unsigned long long eo = block_excl_scan_u64(nout, s, &to);
        if (valid) {
            QueryState &st = b.qs[q];
            st.nsel = nsel;
            st.start = cs + es;
            st.nout = nout;
            st.off = co + eo;
        }
        cs += ts;
        co += to;
    }
    __syncthreads();
    if (tid == 0) {
        if (!selected) b.ctl->nsel = min(b.ctl->npairs, b.rec_cap);
        b.ctl->nout = co;
        const uint32_t db = max(bitlen32(s_dmax), 1u);
        b.ctl->sort_db = db;
        b.ctl->sort_passes = max((qb + db + 2u * vb + 7u) / 8u, 1u);
    }
}

__global__ __launch_bounds__(1024) void k_layout(CallBuffers b, int selected, uint32_t qb, uint32_t vb) {
    __shared__ unsigned long long s[1024];
    __shared__ uint32_t s_dmax;
    layout_block(b, selected, qb, vb, s, s_dmax);
}

// ------------------------------------------------------------------ radix sort
// Records are ordered by the key (q, d, u, v): v in bits [0, vb), u in
// [vb, 2vb), d in [2vb, 2vb + db), q above, sorted by 8-bit digits from the
// least significant, three launches per digit: the per-tile digit histogram,
// its scan, and the stable scatter.  db and the number of digits come from
// the device (k_layout); launches for digits beyond it return at once.
constexpr uint32_t kSortBlocks = 256;
// words of the radix sort's scratch region (per pass a [256 digits][kSortBlocks
// tiles] histogram, then 256 digit totals per pass)
constexpr uint32_t kSortHistWords = (kSortPassesMax + 1) * 256u * (kSortBlocks + 1);

__device__ __forceinline__ void sort_tile(const unsigned long long *nptr, unsigned long long cap,
                                          uint64_t &beg, uint64_t &end, uint64_t &tile) {
    const uint64_t n = min(static_cast<uint64_t>(*nptr), static_cast<uint64_t>(cap));
    tile = (n + gridDim.x - 1) / gridDim.x;
    if (tile == 0) tile = 1;
    beg = min(n, blockIdx.x * tile);
    end = min(n, beg + tile);
}

__device__ __forceinline__ uint32_t rec_digit(const Rec &r, uint32_t bit, uint32_t vb, uint32_t db) {
    const uint32_t sh = 2u * vb;
    const uint64_t lo = (static_cast<uint64_t>(static_cast<uint32_t>(r.u)) << vb) | static_cast<uint32_t>(r.v);
    const uint64_t hi = (static_cast<uint64_t>(r.q) << db) | r.d;
    if (bit >= sh) return static_cast<uint32_t>(hi >> (bit - sh)) & 255u;
    uint64_t x = lo >> bit;
    if (bit + 8u > sh) x |= hi << (sh - bit);
    return static_cast<uint32_t>(x) & 255u;
}

// Stable within-block ranking of one 256-item chunk by an 8-bit digit:
// returns the rank among earlier items with the same digit; wcnt[w][d]
// receives wave w's count of digit d.  Ends with the block synchronised.
__device__ __forceinline__ uint32_t chunk_rank(bool act, uint32_t dg, uint32_t (*wcnt)[256]) {
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    uint64_t peers = __ballot(act);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool set = (dg >> b) & 1u;
        const uint64_t m = __ballot(act && set);
        peers &= set ? m : ~m;
    }
    const uint32_t wrank = mbcnt(peers);
    if (act && wrank == 0) wcnt[wave][dg] = popc(peers);
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < wave; ++w) off += act ? wcnt[w][dg] : 0u;
    return off + wrank;
}

// Exclusive scan over 256 threads (4 waves) through LDS scratch ws[4].
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *ws) {
    const uint32_t tid = threadIdx.x;
    const uint32_t incl = wave_incl_scan(v);
    if ((tid & 63u) == 63u) ws[tid >> 6] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < (tid >> 6); ++w) off += ws[w];
    __syncthreads();
    return off + incl - v;
}

// One pass's digit histogram per tile, laid out [digit][tile], counted in
// LDS over the tile the pass's scatter will read (plain stores: no global
// atomics, whose hot words made passes with a skewed digit up to 15 times
// slower).  Launches beyond ctl->sort_passes return at once.
__global__ __launch_bounds__(256) void k_sort_hist(const Rec *in, const CallCtl *ctl, unsigned long long cap,
                                                   uint32_t vb, uint32_t pass, uint32_t *hist) {
    __shared__ uint32_t h[256];
    if (pass >= ctl->sort_passes) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t beg, end, tile;
    sort_tile(&ctl->nsel, cap, beg, end, tile);
    const uint32_t db = ctl->sort_db;
    for (uint64_t i = beg + threadIdx.x; i < end; i += 256) atomicAdd(&h[rec_digit(in[i], 8u * pass, vb, db)], 1u);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Scan of one pass's histogram: each digit row becomes its exclusive prefix
// over tiles, and tot[d] the row total (one block per digit).
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t *hist, uint32_t *tot, const CallCtl *ctl, uint32_t pass) {
    __shared__ uint32_t ws[4];
    if (pass >= ctl->sort_passes) return;
    const uint32_t d = blockIdx.x, tid = threadIdx.x;
    const uint32_t v = hist[d * kSortBlocks + tid];
    const uint32_t e = block_excl_scan_256(v, ws);
    hist[d * kSortBlocks + tid] = e;
    if (tid == kSortBlocks - 1) tot[d] = e + v;
}

// One digit pass.  hist: this pass's scanned [256][tiles] histogram.  The
// last pass writes each query's first nout records to the caller's buffer at
// the query's offset, when the records all fit and the output fits user_cap.
__global__ __launch_bounds__(256) void k_sort_pass(const Rec *in, Rec *out, CallBuffers b, uint32_t pass,
                                                   uint32_t vb, const uint32_t *hist, const uint32_t *tot,
                                                   rn_pair *user_out,
                                                   unsigned long long user_cap) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t ws[4];
    const uint32_t tid = threadIdx.x;
    const CallCtl *ctl = b.ctl;
    const uint32_t passes = ctl->sort_passes;
    if (pass >= passes) return;
    const bool last = pass + 1 == passes;
    if (last && (ctl->npairs > b.rec_cap || ctl->nout > user_cap)) return;
    const uint32_t db = ctl->sort_db;
    {
        const uint32_t pre = hist[tid * kSortBlocks + blockIdx.x];
        base[tid] = block_excl_scan_256(tot[tid], ws) + pre;
    }
    uint64_t beg, end, tile;
    sort_tile(&ctl->nsel, b.rec_cap, beg, end, tile);
    const uint32_t shift = 8u * pass;
    for (uint64_t c = beg; c < end; c += 256) {
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const uint64_t i = c + tid;
        const bool act = i < end;
        Rec r{0, 0, 0, 0};
        if (act) r = in[i];
        const uint32_t dg = act ? rec_digit(r, shift, vb, db) : 0u;
        const uint32_t pos = base[dg] + chunk_rank(act, dg, wcnt);
        if (act) {
            if (last) {
                const QueryState &st = b.qs[r.q];
                const unsigned long long rel = pos - st.start;
                if (rel < st.nout) {
                    rn_pair p;
                    p.u = r.u;
                    p.v = r.v;
                    p.dist = r.d;
                    user_out[st.off + rel] = p;
                }
            } else {
                out[pos] = r;
            }
        }
        __syncthreads();
        base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

// ---- bucket sort (theta-join calls with few distinct distances per query)
__device__ __forceinline__ uint32_t rec_bin(const CallBuffers &b, const Rec &r) { return b.binbase[r.q] + r.d; }

// One block: bin starts (exclusive prefix of the counts), scatter cursors and
// the first 64-record chunk of each bin; when the chunks fit the radix sort's
// scratch region (unused by this sort), also the bin of every chunk, which
// spares each ranking wave a search over the chunk starts.
__device__ __forceinline__ void bucket_scan_block(const CallBuffers &b, uint32_t *wsum) {
    const uint32_t nb = b.nbins, tid = threadIdx.x;
    const uint32_t *cnt = b.bins;
    uint32_t *start = b.bins + nb, *cursor = b.bins + 2 * nb, *cstart = b.bins + 3 * nb;
    const uint32_t per = (nb + 1023u) / 1024u, lo = min(nb, tid * per), hi = min(nb, lo + per);
    uint32_t sr = 0, sc = 0, big = 0;
    for (uint32_t i = lo; i < hi; ++i) {
        sr += cnt[i];
        sc += (cnt[i] + 63u) / 64u;
        big |= cnt[i] > kBucketRankMax ? 1u : 0u;
    }
    if (big) b.ctl->resort = 1u;   // (the call block starts cleared)
    uint32_t tr, tc;
    uint32_t er = block_excl_scan_1024(sr, wsum, &tr);
    uint32_t ec = block_excl_scan_1024(sc, wsum, &tc);
    const bool map = tc <= kSortHistWords;
    for (uint32_t i = lo; i < hi; ++i) {
        start[i] = er;
        cursor[i] = er + kPlaceNone;   // records past the first kPlaceNone of a bin
        cstart[i] = ec;
        er += cnt[i];
        const uint32_t nch = (cnt[i] + 63u) / 64u;
        if (map)
            for (uint32_t t = 0; t < nch; ++t) b.sort_hist[ec + t] = i;
        ec += nch;
    }
    if (tid == 0) {
        cstart[nb] = tc;
        b.ctl->nchunks = tc;
    }
}

// theta-join calls: the output layout and the bin scan, in one block
__global__ __launch_bounds__(1024) void k_layout_bins(CallBuffers b, uint32_t qb, uint32_t vb) {
    __shared__ unsigned long long s[1024];
    __shared__ uint32_t s_dmax;
    layout_block(b, 0, qb, vb, s, s_dmax);
    __syncthreads();
    bucket_scan_block(b, reinterpret_cast<uint32_t *>(s));
}

// Each record goes to its bin's start plus the place the relaxation kernel's
// bin count gave it (records past the first kPlaceNone of a bin take slots
// from the bin's cursor instead); the query field loses the place again.
__global__ __launch_bounds__(256) void k_bucket_scatter(CallBuffers b) {
    const unsigned long long n = b.ctl->nsel;
    const uint32_t *start = b.bins + b.nbins;
    uint32_t *cursor = b.bins + 2 * b.nbins;
    for (unsigned long long i = blockIdx.x * 256ull + threadIdx.x; i < n; i += gridDim.x * 256ull) {
        Rec r = b.recs[0][i];
        const uint32_t place = r.q >> 16;
        r.q &= 0xFFFFu;
        const uint32_t bin = rec_bin(b, r);
        b.recs[1][place != kPlaceNone ? start[bin] + place : atomicAdd(&cursor[bin], 1u)] = r;
    }
}

// One wave per 64-record chunk of a bin: each record's place in the bin is the
// number of the bin's records with a smaller (u, v) (keys are unique within a
// query); the record goes to the caller's output at its query's offset.  A
// wave's work is the size of its bin, at most kBucketRankMax (beyond it the
// caller takes the radix sort).
__global__ __launch_bounds__(256) void k_bucket_rank(CallBuffers b, rn_pair *out, unsigned long long user_cap,
                                                      const uint32_t *state, uint32_t *state_map, uint32_t state_words) {
    const CallCtl *ctl = b.ctl;
    // the call state is final once the layout has run (the scatter and this
    // ranking only read it): block 0 publishes it, as k_publish does
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < state_words; i += 256) state_map[i] = state[i];
    if (ctl->npairs > b.rec_cap || ctl->nout > user_cap || ctl->resort) return;
    const uint32_t nb = b.nbins, lane = lane_id();
    const uint32_t *cnt = b.bins, *start = b.bins + nb, *cstart = b.bins + 3 * nb;
    const uint32_t total = ctl->nchunks;
    const uint32_t waves = gridDim.x * 4u;
    for (uint32_t c = blockIdx.x * 4u + (threadIdx.x >> 6); c < total; c += waves) {
        const uint32_t bin = total <= kSortHistWords ? b.sort_hist[c] : seg_of(cstart, nb, c);
        const uint32_t m = cnt[bin], s0 = start[bin];
        const uint32_t j = (c - cstart[bin]) * 64u + lane;
        const bool valid = j < m;
        const Rec r = b.recs[1][s0 + (valid ? j : 0u)];
        const uint32_t mu = static_cast<uint32_t>(r.u), mv = static_cast<uint32_t>(r.v);
        uint32_t rank = 0;
        for (uint32_t j0 = 0; j0 < m; j0 += 64u) {
            const uint32_t jj = j0 + lane < m ? j0 + lane : j0;
            const Rec o = b.recs[1][s0 + jj];
            const uint32_t ou = static_cast<uint32_t>(o.u), ov = static_cast<uint32_t>(o.v);
            const uint32_t lim = min(64u, m - j0);
            for (uint32_t t = 0; t < lim; ++t) {
                const uint32_t xu = readlane(ou, static_cast<int>(t)), xv = readlane(ov, static_cast<int>(t));
                rank += (xu < mu || (xu == mu && xv < mv)) ? 1u : 0u;
            }
        }
        if (valid) {
            const QueryState &st = b.qs[r.q];
            const unsigned long long rel = static_cast<unsigned long long>(s0 + rank) - st.start;
            if (rel < st.nout) {
                rn_pair pr;
                pr.u = r.u;
                pr.v = r.v;
                pr.dist = r.d;
                out[st.off + rel] = pr;
            }
        }
    }
}

// ---- small sort (k-closest-pairs calls with few candidates)
// One block: the selected records (recs[1], at most kSmallSort) become 64-bit
// keys (query, dist, u, v) packed as the radix sort orders them (when they fit
// 63 bits), padded with all-ones keys to a power of two and bitonic-sorted in
// LDS (up to three consecutive stages of a merge per barrier, below); the key
// gives the record back, which goes to the caller's output at its query's
// offset.  Too many records or too wide a key: ctl->resort.

// G consecutive stages of bitonic merge k, at compare distances j, j/2, ...,
// j/2^(G-1) = h, over P keys in LDS: the keys at base + m h (m < 2^G, base
// with zero bits where m h sits) meet only each other in those stages, so one
// thread loads the 2^G of them, runs the stages in registers and stores them.
// Whole block; the caller's barrier follows.
template <int G>
__device__ __forceinline__ void bitonic_stages(unsigned long long *s, uint32_t P, uint32_t k, uint32_t j,
                                               uint32_t tid) {
    constexpr uint32_t E = 1u << G;
    const uint32_t h = j >> (G - 1);
    for (uint32_t i = tid; i < P / E; i += 1024) {
        const uint32_t base = ((i & ~(h - 1u)) << G) | (i & (h - 1u));
        const bool up = (base & k) == 0u;   // (the same for the whole group: h * E <= k)
        unsigned long long x[E];
#pragma unroll
        for (uint32_t m = 0; m < E; ++m) x[m] = s[base + m * h];
#pragma unroll
        for (uint32_t d = E / 2; d > 0; d >>= 1) {
#pragma unroll
            for (uint32_t m = 0; m < E; ++m) {
                if ((m & d) != 0u) continue;
                const unsigned long long lo = x[m], hi = x[m + d];
                const bool swap = (lo > hi) == up;
                x[m] = swap ? hi : lo;
                x[m + d] = swap ? lo : hi;
            }
        }
#pragma unroll
        for (uint32_t m = 0; m < E; ++m) s[base + m * h] = x[m];
    }
}

__device__ __forceinline__ void sort_small(const CallBuffers &b, uint32_t qb, uint32_t vb, rn_pair *out,
                                           unsigned long long user_cap, unsigned long long *s_k) {
    CallCtl *ctl = b.ctl;
    if (ctl->npairs > b.rec_cap || ctl->nout > user_cap) return;
    const uint32_t tid = threadIdx.x;
    const unsigned long long n64 = ctl->nsel;
    const uint32_t db = ctl->sort_db;
    if (n64 > kSmallSort || qb + db + 2u * vb > 63u) {
        if (tid == 0) ctl->resort = 1u;
        return;
    }
    const uint32_t n = static_cast<uint32_t>(n64);
    uint32_t P = 2;
    while (P < n) P <<= 1;
    const uint32_t sh_d = 2u * vb, sh_q = 2u * vb + db;
    for (uint32_t i = tid; i < P; i += 1024) {
        unsigned long long key = ~0ull;
        if (i < n) {
            const Rec r = b.recs[1][i];
            key = (static_cast<unsigned long long>(r.q) << sh_q) | (static_cast<unsigned long long>(r.d) << sh_d) |
                  (static_cast<unsigned long long>(static_cast<uint32_t>(r.u)) << vb) | static_cast<uint32_t>(r.v);
        }
        s_k[i] = key;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0;) {
            if (j >= 4) {
                bitonic_stages<3>(s_k, P, k, j, tid);
                j >>= 3;
            } else if (j == 2) {
                bitonic_stages<2>(s_k, P, k, j, tid);
                j >>= 2;
            } else {
                bitonic_stages<1>(s_k, P, k, j, tid);
                j >>= 1;
            }
            __syncthreads();
        }
    }
    const unsigned long long vm = (1ull << vb) - 1ull, dm = (1ull << db) - 1ull;
    for (uint32_t i = tid; i < n; i += 1024) {
        const unsigned long long key = s_k[i];
        const uint32_t q = static_cast<uint32_t>(key >> sh_q);
        const QueryState &st = b.qs[q];
        const unsigned long long rel = static_cast<unsigned long long>(i) - st.start;
        if (rel < st.nout) {
            rn_pair p;
            p.u = static_cast<int32_t>((key >> vb) & vm);
            p.v = static_cast<int32_t>(key & vm);
            p.dist = static_cast<uint32_t>((key >> sh_d) & dm);
            out[st.off + rel] = p;
        }
    }
}

// The output layout of the selected records (as k_layout), the small sort,
// then (every exit of it is block-uniform) the call state's copy into mapped
// host memory, as k_publish does: one launch for what took three.
__global__ __launch_bounds__(1024) void k_sort_small(CallBuffers b, uint32_t qb, uint32_t vb, rn_pair *out,
                                                     unsigned long long user_cap, const uint32_t *state,
                                                     uint32_t *state_map, uint32_t state_words) {
    __shared__ unsigned long long s_k[kSmallSort];
    __shared__ uint32_t s_dmax;
    static_assert(kSmallSort >= 1024, "the layout's scan uses the sort's keys as scratch");
    layout_block(b, 1, qb, vb, s_k, s_dmax);
    __syncthreads();   // the layout's call state (ctl written by thread 0) is seen by the whole block
    sort_small(b, qb, vb, out, user_cap, s_k);
    __syncthreads();   // the state's last writes (ctl->resort) are seen by the whole block
    for (uint32_t i = threadIdx.x; i < state_words; i += 1024) state_map[i] = state[i];
}

// Blocks of `lds` bytes of LDS that one CU holds at once.  A CU's LDS is
// handed out in 128 equal granules (1 280 bytes of the 160 KiB on gfx950), a
// block taking whole granules, while the occupancy query counts bytes: it
// answers 13 for blocks of 12 KiB, of which 12 fit (10 granules each), and a
// persistent grid sized by it leaves the 13th block of every CU waiting for a
// whole block's lifetime.  (Measured with blocks that hold LDS and spin:
// 6 144, 8 192, 12 288 and 16 384 bytes give 25, 18, 12 and 9 blocks; 10 240,
// 11 264, 20 480, 24 576 and 28 672 give what the query says.)
int lds_resident_blocks(size_t lds, size_t lds_per_cu) {
    if (lds == 0 || lds_per_cu < 128) return 1 << 20;
    const size_t gran = lds_per_cu / 128;
    return static_cast<int>(lds_per_cu / ((lds + gran - 1) / gran * gran));
}

template <int HB, bool GEN, bool CT>
hipError_t launch_join_tier(const JoinArgs &a, uint32_t max_sources, bool persistent, hipStream_t s) {
    static int resident = 0;  // blocks per CU, per device this process uses first
    static int cus = 0;
    if (resident == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return e;
        int occ = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_join<HB, GEN, CT>, 64 * Tier<HB, CT>::NW, 0);
        if (e != hipSuccess) return e;
        hipFuncAttributes fa;
        e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_join<HB, GEN, CT>));
        if (e != hipSuccess) return e;
        cus = prop.multiProcessorCount;
        const int fit = lds_resident_blocks(fa.sharedSizeBytes, prop.maxSharedMemoryPerMultiProcessor);
        resident = occ < fit ? occ : fit;
        if (resident < 1) resident = 1;
    }
    // persistent: as many blocks as fit on the device at once, each looping
    // over sources; otherwise one block per source, so that the kernel's
    // blocks are short and launches from other streams interleave with them
    uint64_t grid = static_cast<uint64_t>(cus) * resident;
    grid = (grid + 7) / 8 * 8;
    const uint64_t want = (static_cast<uint64_t>(max_sources) + 7) / 8 * 8;
    if (want < grid || !persistent) grid = want;
    if (grid == 0) grid = 8;
    hipLaunchKernelGGL((k_join<HB, GEN, CT>), dim3(static_cast<uint32_t>(grid)), dim3(64 * Tier<HB, CT>::NW), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_publish(const uint32_t *src, uint32_t *dst, uint32_t words, hipStream_t s) {
    if (words == 0) return hipSuccess;
    const uint32_t blocks = (words + 255u) / 256u;
    hipLaunchKernelGGL(k_publish, dim3(blocks), dim3(256), 0, s, src, dst, words);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

size_t stage_scratch_words(size_t rwords) { return (rwords + 1023) / 1024 + 1; }

hipError_t launch_stage(const CallBuffers &b, unsigned long long max_elems, const int32_t *rank, hipStream_t s) {
    const uint32_t eblk = static_cast<uint32_t>((max_elems + 255) / 256);
    hipLaunchKernelGGL(k_mark, dim3(eblk), dim3(256), 0, s, b, rank);
    const uint32_t nblk = (b.rwords + 1023u) / 1024u;
    const uint32_t oblk = static_cast<uint32_t>((max_elems + 1023) / 1024);
    hipLaunchKernelGGL(k_overlap_count, dim3(max(nblk, oblk)), dim3(1024), 0, s, b, rank, nblk);
    hipLaunchKernelGGL(k_rank_emit, dim3(nblk), dim3(1024), 0, s, b, b.stage_scratch);
    return hipGetLastError();
}

int join_tier_supported(int hash_log2) { return hash_log2 >= kMinHB && hash_log2 <= kMaxHB; }


hipError_t launch_join(const JoinArgs &a, int hash_log2, bool generic, bool compact, uint32_t max_sources,
                       bool persistent, hipStream_t s) {
#define RN_TIER(HB)                                                                                   \
    case HB:                                                                                          \
        if constexpr (HB >= kCompactMinHB) {                                                          \
            if (compact)                                                                              \
                return generic ? launch_join_tier<HB, true, true>(a, max_sources, persistent, s)      \
                               : launch_join_tier<HB, false, true>(a, max_sources, persistent, s);    \
        }                                                                                             \
        return generic ? launch_join_tier<HB, true, false>(a, max_sources, persistent, s)             \
                       : launch_join_tier<HB, false, false>(a, max_sources, persistent, s);
    switch (hash_log2) {
        RN_TIER(8)
        RN_TIER(9)
        RN_TIER(10)
        RN_TIER(11)
        RN_TIER(12)
        RN_TIER(13)
        RN_TIER(14)
        default: return hipErrorInvalidValue;
    }
#undef RN_TIER
}

hipError_t launch_join_global(const JoinArgs &a, uint32_t *slots, uint32_t nslots, int32_t Vmax,
                              uint32_t max_sources, hipStream_t s) {
    uint32_t grid = nslots < max_sources ? nslots : max_sources;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_join_global, dim3(grid), dim3(kGT), 0, s, a, slots, nslots, Vmax);
    return hipGetLastError();
}

hipError_t launch_kcp_seed(const JoinArgs &a, const CallBuffers &b, uint32_t max_sources, hipStream_t s) {
    hipLaunchKernelGGL(k_kcp_seed_hist, dim3((max_sources + 255) / 256), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_kcp_seed_bound, dim3(static_cast<uint32_t>(b.nq)), dim3(64), 0, s, b.qd, b.qs, b.hists,
                       a.count_work ? 0 : 1);
    hipLaunchKernelGGL(k_kcp_direct, dim3((max_sources + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_select(const CallBuffers &b, hipStream_t s) {
    hipLaunchKernelGGL(k_select, dim3(1024), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_layout(const CallBuffers &b, int selected, uint32_t qb, uint32_t vb, bool bins, hipStream_t s) {
    if (bins)
        hipLaunchKernelGGL(k_layout_bins, dim3(1), dim3(1024), 0, s, b, qb, vb);
    else
        hipLaunchKernelGGL(k_layout, dim3(1), dim3(1024), 0, s, b, selected, qb, vb);
    return hipGetLastError();
}

// per pass: a [256 digits][kSortBlocks tiles] histogram, then 256 digit totals per pass
size_t sort_hist_words() { return kSortHistWords; }

hipError_t launch_sort_out(const CallBuffers &b, int selected, uint32_t max_passes, uint32_t vb,
                           rn_pair *out, unsigned long long user_cap, hipStream_t s) {
    if (max_passes > kSortPassesMax) return hipErrorInvalidValue;
    const size_t hw = 256u * kSortBlocks;
    uint32_t *hist = b.sort_hist;
    uint32_t *tot = hist + (kSortPassesMax + 1) * hw;
    Rec *in = selected ? b.recs[1] : b.recs[0];
    Rec *o = selected ? b.recs[0] : b.recs[1];
    for (uint32_t p = 0; p < max_passes; ++p) {
        hipLaunchKernelGGL(k_sort_hist, dim3(kSortBlocks), dim3(256), 0, s, in, b.ctl, b.rec_cap, vb, p, hist + p * hw);
        hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(256), 0, s, hist + p * hw, tot + p * 256u, b.ctl, p);
        hipLaunchKernelGGL(k_sort_pass, dim3(kSortBlocks), dim3(256), 0, s, in, o, b, p, vb, hist + p * hw,
                           tot + p * 256u, out, user_cap);
        Rec *t = in;
        in = o;
        o = t;
    }
    return hipGetLastError();
}

hipError_t launch_sort_small(const CallBuffers &b, uint32_t qb, uint32_t vb, rn_pair *out, unsigned long long user_cap,
                             const uint32_t *state, uint32_t *state_map, uint32_t state_words, hipStream_t s) {
    hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(1024), 0, s, b, qb, vb, out, user_cap, state, state_map,
                       state_words);
    return hipGetLastError();
}

hipError_t launch_bucket_sort(const CallBuffers &b, rn_pair *out, unsigned long long user_cap, const uint32_t *state,
                              uint32_t *state_map, uint32_t state_words, hipStream_t s) {
    hipLaunchKernelGGL(k_bucket_scatter, dim3(1024), dim3(256), 0, s, b);
    hipLaunchKernelGGL(k_bucket_rank, dim3(1024), dim3(256), 0, s, b, out, user_cap, state, state_map, state_words);
    return hipGetLastError();
}

}  // namespace rn
