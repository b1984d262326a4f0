// rn_kernels.hip -- gfx950 kernels of the network-distance joins.
//
// Query pipeline (one HIP stream, no host round trip in between):
//   stage     validate R and S, build the S-membership bitmap and the ordered
//             source list (k_mark, k_overlap, k_compact)
//   relax     one wavefront per source: a bounded, bucketed label-correcting
//             search whose whole state (distance table, pending set, frontier)
//             lives in LDS; emits (u, v, dist) for v in S (k_join)
//   sort      LSD radix sort of the pairs on the (dist, u, v) key
//   copy-out  into the caller's buffer when the query succeeded and fits
//
// The queries are the paper's theta-join and k-closest pairs (Abstract;
// Section 1; Section 4).  The per-source search plays the role of the paper's
// local best-first search from each w in R that tests every reached node for
// membership in S (Section 4, the text after Algorithm 3); here it is not
// confined to a partition, so no cross-edge expansion (Algorithms 3-4) is
// needed and the result is exact.
#include <hip/hip_runtime.h>

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
// 3/4).  PC: capacity of each vertex list (pending set, frontier).
template <int HB>
struct Tier {
    static constexpr int H = 1 << HB;
    static constexpr int PC = HB <= 9 ? 128 : (HB <= 11 ? 256 : (HB == 12 ? 512 : 1024));
    static constexpr int U = (H / 64) < 8 ? (H / 64) : 8;   // table rows scanned per batch
};

// Distance words: (distance << 1) | pending, the low bit set while the vertex
// is in the pending list.  One atomicMin with (nd << 1) | 1 lowers the distance
// and marks the vertex pending only when nd is strictly smaller (an equal
// distance over a zero-weight arc leaves the word alone); the lane that finds
// the old word idle or empty appends the vertex.  Expansion clears the bit.
// On-chip tables therefore hold distances up to 2^31 - 2; a search that needs
// longer ones moves on to the global tier.
constexpr uint32_t kWordNone = 0xFFFFFFFFu;   // empty slot (above every stored word)
constexpr uint32_t kPackMax = 0x7FFFFFFEu;    // largest distance an on-chip table holds
constexpr uint32_t kNoKey = 0xFFFFFFFEu;      // compare value no stored key equals

template <int HB>
struct SearchLds {
    static constexpr int H = Tier<HB>::H;
    static constexpr int PC = Tier<HB>::PC;
    uint32_t key[H];            // vertex id, or kEmpty
    uint32_t dw[H];             // distance word, kWordNone when empty
    uint32_t ent[2][PC + 1];    // two vertex lists: slot | (arc count << 16) and first arc;
    int32_t beg[2][PC + 1];     //   entry PC of each is a write sink for lanes with nothing to store
    int32_t widx[kWin];         // window arc -> arc index
    uint32_t wd[kWin];          // window arc -> distance of the arc's tail
};

struct WaveState {
    uint32_t np;    // entries in the pending list
    uint32_t nins;  // table entries in use
    uint32_t imin;  // per-lane min of the distances improved this phase
    bool ovf;       // the search outgrew this tier
};

__device__ __forceinline__ uint32_t current_bound(const JoinArgs &a) {
    if (!a.kcp) return a.theta;
    uint32_t t = __hip_atomic_load(&a.ctl->theta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return min(t, a.theta);
}

// Relax NJ window arcs per lane (slot j holds window arc j*64 + lane) and
// append targets that became pending to list P.  Two LDS steps, each issued
// for all NJ slots before any result is used: claim-or-find the target's slot
// (compare-and-swap on an empty home slot doubles as the first probe), then
// the packed atomicMin.  Idle lanes issue no-op atomics instead of branching.
// Called by all 64 lanes; st.ovf is wave-uniform afterwards.
template <int HB, int NJ>
__device__ __forceinline__ void relax_window(SearchLds<HB> &L, WaveState &st, uint32_t P,
                                             const ArcRec *r, const uint32_t *nd, uint32_t bound) {
    constexpr uint32_t H = Tier<HB>::H;
    constexpr uint32_t PC = Tier<HB>::PC;
    // slot states: 0 idle, 1 slot holds y, 2 slot claimed for y, 3 keep probing
    uint32_t h[NJ], stt[NJ], old[NJ];
    bool big = false;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        // idle lanes aim their no-op atomics at distinct slots: a shared address would serialise
        h[j] = nd[j] <= bound ? slot_hash<HB>(static_cast<uint32_t>(r[j].y)) : lane_id();
        big |= nd[j] <= bound && nd[j] > kPackMax;
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        old[j] = atomicCAS(&L.key[h[j]], nd[j] <= bound ? kEmpty : kNoKey, static_cast<uint32_t>(r[j].y));
    bool probe = false;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint32_t y = static_cast<uint32_t>(r[j].y);
        stt[j] = nd[j] > bound ? 0u : (old[j] == kEmpty ? 2u : (old[j] == y ? 1u : 3u));
        probe |= stt[j] == 3u;
    }
    bool lost = big;
    if (__ballot(probe) != 0) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            if (stt[j] == 3u) {  // linear probing past an occupied home slot
                const uint32_t y = static_cast<uint32_t>(r[j].y);
                uint32_t hh = h[j];
                for (uint32_t q = 1; q < H; ++q) {
                    hh = (hh + 1) & (H - 1);
                    const uint32_t o = atomicCAS(&L.key[hh], kEmpty, y);
                    if (o == kEmpty) { stt[j] = 2u; break; }
                    if (o == y) { stt[j] = 1u; break; }
                }
                if (stt[j] == 3u) lost = true;
                h[j] = hh;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint32_t v =
            (stt[j] == 1u || stt[j] == 2u) && nd[j] <= kPackMax ? (nd[j] << 1) | 1u : kWordNone;
        old[j] = atomicMin(&L.dw[h[j]], v);
        // 4: improved a pending vertex; 5: improved an idle or new one, which this lane appends
        stt[j] = (v < old[j]) ? ((old[j] == kWordNone || (old[j] & 1u) == 0u) ? 5u : 4u) : stt[j];
    }
    uint64_t mA[NJ];
    uint32_t nadd = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const bool imp = stt[j] >= 4u;
        st.imin = min(st.imin, imp ? nd[j] : kInf);
        mA[j] = __ballot(stt[j] == 5u);
        nadd += popc(mA[j]);
        lost |= stt[j] == 5u && (r[j].yend - r[j].ybeg) > 0xFFFF;
    }
    uint32_t ins = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) ins += popc(__ballot(old[j] == kWordNone && stt[j] >= 4u));
    st.nins += ins;
    if (__ballot(lost) != 0 || st.nins > (3u * H) / 4u || st.np + nadd > PC) {
        st.ovf = true;
        return;
    }
    uint32_t base = st.np;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const bool app = stt[j] == 5u;
        const uint32_t idx = app ? base + mbcnt(mA[j]) : PC;
        L.ent[P][idx] = h[j] | (static_cast<uint32_t>(r[j].yend - r[j].ybeg) << 16);
        L.beg[P][idx] = r[j].ybeg;
        base += popc(mA[j]);
    }
    st.np = base;
}

// Load window arcs j*64 + lane (j < NJ) and relax them.  Every load is issued
// before any is used; lanes past the window's end load arc 0 and stay idle.
template <int HB, int NJ>
__device__ __forceinline__ void window_step(SearchLds<HB> &L, WaveState &st, uint32_t P,
                                            const ArcRec *__restrict__ arcs, uint32_t cnt,
                                            uint32_t bound) {
    const uint32_t lane = lane_id();
    int32_t idx[NJ];
    uint32_t od[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const uint32_t t = j * 64 + lane;
        const uint32_t tc = t < cnt ? t : 0u;
        idx[j] = t < cnt ? L.widx[tc] : 0;
        od[j] = L.wd[tc];
    }
    ArcRec r[NJ];
    uint32_t nd[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) r[j] = arcs[idx[j]];
#pragma unroll
    for (int j = 0; j < NJ; ++j) nd[j] = (j * 64 + lane < cnt) ? sat_add(od[j], r[j].w) : kInf;
    wave_sync();  // window map fully read before the next window rewrites it
    relax_window<HB, NJ>(L, st, P, r, nd, bound);
}

// k-closest pairs: once k pairs have been emitted, bound the k-th distance by
// the emitted-distance histogram and lower the shared bound.  Whole wave.
__device__ __forceinline__ void tighten_bound(const JoinArgs &a) {
    const unsigned long long n =
        __hip_atomic_load(&a.ctl->npairs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n < a.k) return;
    const uint32_t b = wave_bound_from_hist(a.cand_hist, a.k);
    if ((threadIdx.x & 63u) == 0) atomicMin(&a.ctl->theta, b);
}

// Write this wave's staged pairs (v in L.beg[0], dist in L.ent[0]) for source u.
template <int HB>
__device__ __forceinline__ void flush_pairs(SearchLds<HB> &L, const JoinArgs &a, int32_t u,
                                            uint32_t &nst) {
    if (nst == 0) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&a.ctl->npairs, static_cast<unsigned long long>(nst));
    base = (static_cast<unsigned long long>(readlane(static_cast<uint32_t>(base >> 32), 0)) << 32) |
           readlane(static_cast<uint32_t>(base), 0);
    wave_sync();
    for (uint32_t i = lane_id(); i < nst; i += 64) {
        const unsigned long long idx = base + i;
        if (idx < a.pair_cap) {
            rn_pair p;
            p.u = u;
            p.v = L.beg[0][i];
            p.dist = L.ent[0][i];
            a.pairs[idx] = p;
        }
    }
    wave_sync();
    nst = 0;
}

// Bounded search from u.  Bucket b holds tentative distances in
// [b*delta, (b+1)*delta); each phase expands every pending vertex of the
// lowest non-empty bucket and relaxes its arcs.  With delta <= the smallest
// arc weight each vertex is expanded once, at its final distance (Dijkstra
// order by buckets); a larger delta trades re-expansions for fewer phases, and
// delta = 0 expands the whole pending set every phase (the pending list simply
// becomes the next frontier).  A vertex's distance is read when its frontier
// chunk is expanded, so improvements made earlier in the same phase are used
// at once.  The search ends when nothing is pending; every table entry then
// holds its exact distance, and entries in S become pairs.
template <int HB>
__device__ void search_source(SearchLds<HB> &L, const JoinArgs &a, int32_t u) {
    constexpr int H = Tier<HB>::H;
    constexpr int PC = Tier<HB>::PC;
    constexpr int U = Tier<HB>::U;
    const uint32_t lane = lane_id();
    const int32_t ub = a.row_ptr[u];
    const int32_t ue = a.row_ptr[u + 1];
    if (lane == 0) {
        const uint32_t h0 = slot_hash<HB>(static_cast<uint32_t>(u));   // table is empty
        lds_store(&L.key[h0], static_cast<uint32_t>(u));
        L.dw[h0] = 1u;                                                // distance 0, pending
        L.ent[0][0] = h0 | (static_cast<uint32_t>(min(ue - ub, 0xFFFF)) << 16);
        L.beg[0][0] = ub;
    }
    wave_sync();
    WaveState st;
    st.np = 1;
    st.nins = 1;
    st.ovf = (ue - ub) > 0xFFFF;
    uint32_t P = 0;      // list receiving appends (the pending list)
    uint32_t pmin = 0;
    uint32_t bound = a.theta;

    while (st.np > 0 && !st.ovf) {
        bound = current_bound(a);
        uint32_t F, nf;
        uint32_t kmin = kInf;
        if (a.delta == 0) {
            F = P;
            nf = st.np;
            P ^= 1u;
            st.np = 0;
        } else {
            const uint64_t t64 = (static_cast<uint64_t>(pmin / a.delta) + 1ull) * a.delta;
            const uint32_t thr = t64 > kInf ? kInf : static_cast<uint32_t>(t64);
            F = P ^ 1u;
            nf = 0;
            uint32_t nk = 0;
            for (uint32_t base = 0; base < st.np; base += 64) {
                const uint32_t i = base + lane;
                const bool valid = i < st.np;
                const uint32_t ic = valid ? i : 0u;
                const uint32_t e = L.ent[P][ic];
                const int32_t b = L.beg[P][ic];
                const uint32_t d = L.dw[e & 0xFFFFu] >> 1;
                const bool isF = valid && d < thr && d <= bound;
                const bool isK = valid && d >= thr && d <= bound;
                const bool drop = valid && d > bound;
                const uint64_t mF = __ballot(isF), mK = __ballot(isK);
                wave_sync();  // every lane has read its entry before the in-place compaction
                atomicAnd(&L.dw[valid ? (e & 0xFFFFu) : lane], drop ? ~1u : 0xFFFFFFFFu);  // dropped: not pending
                const uint32_t fi = isF ? nf + mbcnt(mF) : static_cast<uint32_t>(PC);
                L.ent[F][fi] = e;
                L.beg[F][fi] = b;
                const uint32_t ki = isK ? nk + mbcnt(mK) : static_cast<uint32_t>(PC);
                L.ent[P][ki] = e;
                L.beg[P][ki] = b;
                kmin = min(kmin, isK ? d : kInf);
                nf += popc(mF);
                nk += popc(mK);
            }
            st.np = nk;
        }
        st.imin = kInf;
        wave_sync();
        // ---- expand the frontier, kWin arcs at a time
        for (uint32_t fb = 0; fb < nf && !st.ovf; fb += 64) {
            const uint32_t f = fb + lane;
            const bool valid = f < nf;
            const uint32_t fc = valid ? f : 0u;
            const uint32_t e = L.ent[F][fc];
            const int32_t b = L.beg[F][fc];
            const uint32_t s = e & 0xFFFFu;
            const uint32_t d = L.dw[s] >> 1;
            atomicAnd(&L.dw[valid ? s : lane], valid ? ~1u : 0xFFFFFFFFu);  // expanded now: not pending
            const uint32_t deg = (valid && d <= bound) ? (e >> 16) : 0u;
            const uint32_t incl = wave_incl_scan(deg);
            const uint32_t excl = incl - deg;
            const uint32_t total = readlane(incl, 63);
            for (uint32_t wb = 0; wb < total && !st.ovf; wb += kWin) {
                const uint32_t lo = max(excl, wb), hi = min(excl + deg, wb + kWin);
                for (uint32_t p = lo; p < hi; ++p) {
                    L.widx[p - wb] = b + static_cast<int32_t>(p - excl);
                    L.wd[p - wb] = d;
                }
                wave_sync();
                const uint32_t cnt = min(kWin, total - wb);
                switch ((cnt + 63u) / 64u) {
                    case 1: window_step<HB, 1>(L, st, P, a.arcs, cnt, bound); break;
                    case 2: window_step<HB, 2>(L, st, P, a.arcs, cnt, bound); break;
                    case 3: window_step<HB, 3>(L, st, P, a.arcs, cnt, bound); break;
                    default: window_step<HB, 4>(L, st, P, a.arcs, cnt, bound); break;
                }
                wave_sync();
            }
        }
        if (st.ovf) break;
        if (a.delta != 0) pmin = min(wave_min(kmin), wave_min(st.imin));
    }

    // ---- emit table entries in S, and clear the table for the next source
    bound = current_bound(a);
    uint32_t nst = 0, emitted = 0;
    unsigned long long warcs = 0;
    uint32_t wsettled = 0;
    for (uint32_t g0 = 0; g0 < static_cast<uint32_t>(H); g0 += 64 * U) {
        uint32_t k[U], d[U], sb[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t slot = g0 + j * 64 + lane;
            k[j] = lds_load(&L.key[slot]);
            d[j] = L.dw[slot] >> 1;
            sb[j] = 0;
            if (!st.ovf && k[j] != kEmpty) sb[j] = a.sbits[k[j] >> 5];
        }
        if (a.count_work && !st.ovf) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (k[j] != kEmpty && d[j] <= bound) {
                    warcs += static_cast<unsigned long long>(a.row_ptr[k[j] + 1] - a.row_ptr[k[j]]);
                    wsettled += 1;
                }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t slot = g0 + j * 64 + lane;
            lds_store(&L.key[slot], kEmpty);
            L.dw[slot] = kWordNone;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t y = k[j];
            const bool m = !st.ovf && y != kEmpty && ((sb[j] >> (y & 31u)) & 1u) && d[j] <= bound;
            const uint64_t mM = __ballot(m);
            if (a.kcp && m) atomicAdd(&a.cand_hist[dist_bin(d[j])], 1u);
            emitted += popc(mM);
            const uint32_t idx = m ? nst + mbcnt(mM) : static_cast<uint32_t>(PC);
            L.beg[0][idx] = static_cast<int32_t>(y);
            L.ent[0][idx] = d[j];
            nst += popc(mM);
            if (nst + 64 > static_cast<uint32_t>(PC)) {
                wave_sync();
                flush_pairs<HB>(L, a, u, nst);
            }
        }
    }
    wave_sync();
    flush_pairs<HB>(L, a, u, nst);
    if (a.kcp && emitted != 0) tighten_bound(a);
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
        a.ovf[idx] = static_cast<uint32_t>(u);
    }
    wave_sync();
}

// One wavefront per block; sources split into 8 contiguous chunks, chunk c
// taken by the blocks with blockIdx % 8 == c so that each XCD (blocks are
// dealt to the 8 XCDs round-robin) sweeps one region of the source order and
// keeps its part of the graph in its own L2.
template <int HB>
__global__ __launch_bounds__(64) void k_join(JoinArgs a) {
    __shared__ SearchLds<HB> L;
    constexpr int H = Tier<HB>::H;
    const uint32_t n = *a.nsrc;
    const uint32_t per = (n + 7u) / 8u;
    if (blockIdx.x >= 8u * per) return;
    for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(H); i += 64) {
        lds_store(&L.key[i], kEmpty);
        L.dw[i] = kWordNone;
    }
    wave_sync();
    for (uint32_t t = blockIdx.x; t < 8u * per; t += gridDim.x) {
        const uint32_t si = (t & 7u) * per + (t >> 3);
        if (si >= n) continue;
        search_source<HB>(L, a, a.src[si]);
    }
}

// ------------------------------------------------------------------ global-memory tier
// A search that outgrows every on-chip table runs here: one 256-thread block
// per source, its distances in a dense per-slot array, frontier-synchronous
// (every vertex improved in a round is expanded in the next).  Only rare, very
// large searches (huge balls, expander graphs, unbounded k-closest-pairs
// searches) take this path.
__device__ __forceinline__ uint32_t gload(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gstore(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) void k_join_global(JoinArgs a, uint32_t *slots, size_t slot_words,
                                                     int32_t V) {
    __shared__ uint32_t s_nf, s_nfn, s_ntouched, s_bound;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t n = *a.nsrc;
    const size_t nw = (static_cast<size_t>(V) + 31) / 32;
    uint32_t *dist = slots + blockIdx.x * slot_words;
    uint32_t *inq = dist + V;
    uint32_t *fa = inq + nw;
    uint32_t *fb = fa + V;
    uint32_t *touched = fb + V;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int32_t u = a.src[i];
        if (tid == 0) {
            gstore(&dist[u], 0u);
            fa[0] = static_cast<uint32_t>(u);
            touched[0] = static_cast<uint32_t>(u);
            s_nf = 1;
            s_ntouched = 1;
        }
        __syncthreads();
        uint32_t *F = fa, *Fn = fb;
        while (true) {
            const uint32_t nf = s_nf;
            if (nf == 0) break;
            __syncthreads();
            if (tid == 0) {
                s_nfn = 0;
                s_bound = current_bound(a);
            }
            for (uint32_t j = tid; j < nf; j += 256) {
                const uint32_t x = F[j];
                atomicAnd(&inq[x >> 5], ~(1u << (x & 31u)));
            }
            __syncthreads();
            const uint32_t bound = s_bound;
            for (uint32_t j = tid; j < nf; j += 256) {
                const uint32_t x = F[j];
                const uint32_t dx = gload(&dist[x]);
                if (dx > bound) continue;
                const int32_t e = a.row_ptr[x + 1];
                for (int32_t arc = a.row_ptr[x]; arc < e; ++arc) {
                    const ArcRec r = a.arcs[arc];
                    const uint32_t nd = sat_add(dx, r.w);
                    if (nd > bound) continue;
                    const uint32_t y = static_cast<uint32_t>(r.y);
                    const uint32_t old = atomicMin(&dist[y], nd);
                    if (nd >= old) continue;
                    if (old == kInf) touched[atomicAdd(&s_ntouched, 1u)] = y;
                    const uint32_t bit = 1u << (y & 31u);
                    if ((atomicOr(&inq[y >> 5], bit) & bit) == 0) Fn[atomicAdd(&s_nfn, 1u)] = y;
                }
            }
            __syncthreads();
            if (tid == 0) s_nf = s_nfn;
            __syncthreads();
            uint32_t *t = F;
            F = Fn;
            Fn = t;
        }
        // emit S members, count work, reset the slot
        if (tid == 0) s_bound = current_bound(a);
        __syncthreads();
        const uint32_t bound = s_bound;
        const uint32_t nt = s_ntouched;
        unsigned long long warcs = 0;
        uint32_t wsettled = 0;
        for (uint32_t j0 = 0; j0 < nt; j0 += 256) {
            const uint32_t j = j0 + tid;
            uint32_t y = 0, d = kInf;
            bool m = false;
            if (j < nt) {
                y = touched[j];
                d = gload(&dist[y]);
                gstore(&dist[y], kInf);
                m = d <= bound && ((a.sbits[y >> 5] >> (y & 31u)) & 1u);
                if (a.count_work && d <= bound) {
                    warcs += static_cast<unsigned long long>(a.row_ptr[y + 1] - a.row_ptr[y]);
                    wsettled += 1;
                }
            }
            const uint64_t mm = __ballot(m);
            if (a.kcp && m) atomicAdd(&a.cand_hist[dist_bin(d)], 1u);
            if (mm != 0) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(&a.ctl->npairs, static_cast<unsigned long long>(popc(mm)));
                const uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(base & 0xFFFFFFFFull), 0));
                const uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(base >> 32), 0));
                base = (static_cast<unsigned long long>(hi) << 32) | lo;
                const unsigned long long idx = base + mbcnt(mm);
                if (m && idx < a.pair_cap) {
                    rn_pair p;
                    p.u = u;
                    p.v = static_cast<int32_t>(y);
                    p.dist = d;
                    a.pairs[idx] = p;
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
        if (a.kcp && tid < 64) tighten_bound(a);
    }
}

// ------------------------------------------------------------------ staging
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_mark(const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, int32_t V,
                       const int32_t *rank, uint32_t *rbits, uint32_t *sbits, QueryCtl *ctl) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i < nS) {
        const int32_t s = S[i];
        if (s < 0 || s >= V) { atomicOr(&ctl->err, kErrRange); return; }
        const uint32_t bit = 1u << (s & 31);
        if (atomicOr(&sbits[s >> 5], bit) & bit) atomicOr(&ctl->err, kErrDupS);
    } else if (i < static_cast<int64_t>(nS) + nR) {
        const int32_t u = R[i - nS];
        if (u < 0 || u >= V) { atomicOr(&ctl->err, kErrRange); return; }
        const int32_t r = rank ? rank[u] : u;
        const uint32_t bit = 1u << (r & 31);
        if (atomicOr(&rbits[r >> 5], bit) & bit) atomicOr(&ctl->err, kErrDupR);
    }
}

__global__ void k_overlap(const int32_t *R, int32_t nR, int32_t V, const uint32_t *sbits,
                          QueryCtl *ctl) {
    const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    if (i >= nR) return;
    const int32_t u = R[i];
    if (u >= 0 && u < V && ((sbits[u >> 5] >> (u & 31)) & 1u)) atomicOr(&ctl->err, kErrOverlap);
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

// Source listing, pass 1: marked ranks per 1024-word block of the rank bitmap.
__global__ __launch_bounds__(1024) void k_rank_count(const uint32_t *rbits, uint32_t nwords,
                                                     uint32_t *bsum) {
    __shared__ uint32_t wsum[16];
    const uint32_t i = blockIdx.x * 1024u + threadIdx.x;
    uint32_t total;
    block_excl_scan_1024(i < nwords ? __popc(rbits[i]) : 0u, wsum, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Source listing, pass 2: list the marked ranks in increasing order as vertex ids.
__global__ __launch_bounds__(1024) void k_rank_emit(const uint32_t *rbits, uint32_t nwords,
                                                    const uint32_t *bsum, const int32_t *order,
                                                    int32_t *src, QueryCtl *ctl) {
    __shared__ uint32_t wsum[16];
    const uint32_t tid = threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t j = tid; j < blockIdx.x; j += 1024) acc += bsum[j];
    uint32_t pre;
    block_excl_scan_1024(acc, wsum, &pre);
    const uint32_t i = blockIdx.x * 1024u + tid;
    uint32_t bits = i < nwords ? rbits[i] : 0u;
    uint32_t total;
    uint32_t pos = pre + block_excl_scan_1024(__popc(bits), wsum, &total);
    while (bits) {
        const uint32_t b = __ffs(bits) - 1u;
        const int32_t r = static_cast<int32_t>(i * 32u + b);
        src[pos++] = order ? order[r] : r;
        bits &= bits - 1u;
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) ctl->nsrc = pre + total;
}

// ------------------------------------------------------------------ radix sort
// Pairs are ordered by the key (dist, u, v).  When dist and the two ids fit in
// 64 bits the pairs are packed into uint64 keys dist:u:v (vb bits per id) and
// sorted by 8-bit digits, two launches per digit: a scan of the per-tile
// digit histogram (which the previous pass accumulated for the tiles its items
// landed in) and the stable scatter.  Otherwise a three-launch-per-digit sort
// of the 12-byte records is used.
constexpr uint32_t kSortBlocks = 256;
constexpr uint32_t kSortPassesMax = 8;

__device__ __forceinline__ void sort_tile(const unsigned long long *nptr, unsigned long long cap,
                                          uint64_t &beg, uint64_t &end, uint64_t &tile) {
    const uint64_t n = min(static_cast<uint64_t>(*nptr), static_cast<uint64_t>(cap));
    tile = (n + gridDim.x - 1) / gridDim.x;
    if (tile == 0) tile = 1;
    beg = min(n, blockIdx.x * tile);
    end = min(n, beg + tile);
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

// Scan of one pass's histogram, laid out [digit][tile]: each row becomes its
// exclusive prefix over tiles, and tot[d] the row total (one block per digit).
__global__ __launch_bounds__(256) void k_sort_scan(uint32_t *hist, uint32_t *tot) {
    __shared__ uint32_t ws[4];
    const uint32_t d = blockIdx.x, tid = threadIdx.x;
    const uint32_t v = hist[d * kSortBlocks + tid];
    const uint32_t e = block_excl_scan_256(v, ws);
    hist[d * kSortBlocks + tid] = e;
    if (tid == kSortBlocks - 1) tot[d] = e + v;
}

// This block's first output position for each digit (thread d computes digit d)
// from the scanned histogram row and the digit totals.
__device__ __forceinline__ uint32_t digit_start(const uint32_t *hist, const uint32_t *tot, uint32_t *ws) {
    const uint32_t tid = threadIdx.x;
    const uint32_t pre = hist[tid * kSortBlocks + blockIdx.x];
    return block_excl_scan_256(tot[tid], ws) + pre;
}

__device__ __forceinline__ uint64_t pack_pair(const rn_pair &p, uint32_t vb) {
    return (static_cast<uint64_t>(p.dist) << (2u * vb)) |
           (static_cast<uint64_t>(static_cast<uint32_t>(p.u)) << vb) | static_cast<uint32_t>(p.v);
}

__global__ __launch_bounds__(256) void k_sort_pack(const rn_pair *in, uint64_t *keys,
                                                   const unsigned long long *nptr, unsigned long long cap,
                                                   uint32_t vb, uint32_t *hist0) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t beg, end, tile;
    sort_tile(nptr, cap, beg, end, tile);
    for (uint64_t i = beg + threadIdx.x; i < end; i += 256) {
        const uint64_t k = pack_pair(in[i], vb);
        keys[i] = k;
        atomicAdd(&h[k & 255u], 1u);
    }
    __syncthreads();
    hist0[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// One digit pass.  hist: [256][gridDim] counts of this pass's digit per input
// tile.  hist_next (or null): accumulates the next digit per output tile.
// out_pairs (final pass only): receives the unpacked pairs, written only when
// the query succeeded and its result fits.
__global__ __launch_bounds__(256) void k_sort_pass(const uint64_t *in, uint64_t *out, rn_pair *out_pairs,
                                                   const unsigned long long *nptr, unsigned long long cap,
                                                   uint32_t shift, uint32_t vb, const uint32_t *hist,
                                                   const uint32_t *tot, uint32_t *hist_next, uint32_t next_shift,
                                                   const QueryCtl *ctl, unsigned long long user_cap,
                                                   unsigned long long out_limit, int last_tier) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t ws[4];
    const uint32_t tid = threadIdx.x, nb = gridDim.x;
    if (out_pairs) {
        const unsigned long long n = *nptr;
        if (ctl->err != 0 || n > cap || min(n, out_limit) > user_cap) return;
        if (last_tier >= 0 && ctl->novf[last_tier] != 0) return;
    }
    base[tid] = digit_start(hist, tot, ws);
    uint64_t beg, end, tile;
    sort_tile(nptr, cap, beg, end, tile);
    const uint32_t mask = (1u << vb) - 1u;
    for (uint64_t c = beg; c < end; c += 256) {
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const uint64_t i = c + tid;
        const bool act = i < end;
        const uint64_t k = act ? in[i] : 0ull;
        const uint32_t dg = static_cast<uint32_t>(k >> shift) & 255u;
        const uint32_t r = chunk_rank(act, dg, wcnt);
        if (act) {
            const uint32_t pos = base[dg] + r;
            if (out_pairs) {
                rn_pair p;
                p.dist = static_cast<uint32_t>(k >> (2u * vb));
                p.u = static_cast<int32_t>(static_cast<uint32_t>(k >> vb) & mask);
                p.v = static_cast<int32_t>(static_cast<uint32_t>(k) & mask);
                if (pos < out_limit) out_pairs[pos] = p;
            } else {
                out[pos] = k;
            }
            if (hist_next)
                atomicAdd(&hist_next[(static_cast<uint32_t>(k >> next_shift) & 255u) * nb +
                                     pos / static_cast<uint32_t>(tile)],
                          1u);
        }
        __syncthreads();
        base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

// ---- generic path: 12-byte records, any key width
__device__ __forceinline__ uint32_t pair_digit(const rn_pair &p, uint32_t bit, uint32_t vb) {
    const uint32_t sh = 2u * vb;
    if (bit >= sh) return (p.dist >> (bit - sh)) & 255u;
    const uint64_t lo = (static_cast<uint64_t>(static_cast<uint32_t>(p.u)) << vb) |
                        static_cast<uint32_t>(p.v);
    uint64_t x = lo >> bit;
    if (bit + 8u > sh) x |= static_cast<uint64_t>(p.dist) << (sh - bit);
    return static_cast<uint32_t>(x) & 255u;
}

__global__ __launch_bounds__(256) void k_radix_hist(const rn_pair *in, const unsigned long long *nptr,
                                                    unsigned long long cap, uint32_t bit,
                                                    uint32_t vb, uint32_t *hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t beg, end, tile;
    sort_tile(nptr, cap, beg, end, tile);
    for (uint64_t i = beg + threadIdx.x; i < end; i += 256) atomicAdd(&h[pair_digit(in[i], bit, vb)], 1u);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_radix_scatter(const rn_pair *in, rn_pair *out,
                                                       const unsigned long long *nptr,
                                                       unsigned long long cap, uint32_t bit,
                                                       uint32_t vb, const uint32_t *hist,
                                                       const uint32_t *tot) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t ws[4];
    const uint32_t tid = threadIdx.x;
    base[tid] = digit_start(hist, tot, ws);
    uint64_t beg, end, tile;
    sort_tile(nptr, cap, beg, end, tile);
    for (uint64_t c = beg; c < end; c += 256) {
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const uint64_t i = c + tid;
        const bool act = i < end;
        rn_pair p{0, 0, 0};
        if (act) p = in[i];
        const uint32_t dg = act ? pair_digit(p, bit, vb) : 0u;
        const uint32_t r = chunk_rank(act, dg, wcnt);
        if (act) out[base[dg] + r] = p;
        __syncthreads();
        base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

__global__ void k_copy_out(const rn_pair *src, rn_pair *dst, const unsigned long long *nptr,
                           const QueryCtl *ctl, unsigned long long user_cap, unsigned long long limit,
                           unsigned long long out_limit, int last_tier) {
    const unsigned long long n = *nptr;
    if (ctl->err != 0 || n > limit || min(n, out_limit) > user_cap) return;
    if (last_tier >= 0 && ctl->novf[last_tier] != 0) return;
    const unsigned long long m = min(n, out_limit);
    for (unsigned long long i = blockIdx.x * static_cast<unsigned long long>(blockDim.x) + threadIdx.x;
         i < m; i += static_cast<unsigned long long>(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

// ------------------------------------------------------------------ k-closest pairs
// Seed: every distinct (u, y) with u in R, y in S joined by an arc has
// dist(u, y) <= the lightest such arc's weight, so the bin edge where k of
// these weights are reached bounds the k-th smallest distance.  A pair with
// parallel arcs is counted once, at its first lightest arc.
__global__ void k_kcp_seed_hist(const int32_t *src, const uint32_t *nsrc, const int32_t *row_ptr,
                                const ArcRec *arcs, const uint32_t *sbits, uint32_t *seed_hist) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *nsrc) return;
    const int32_t u = src[i];
    const int32_t b = row_ptr[u], e = row_ptr[u + 1];
    for (int32_t x = b; x < e; ++x) {
        const ArcRec r = arcs[x];
        const uint32_t y = static_cast<uint32_t>(r.y);
        if (!((sbits[y >> 5] >> (y & 31u)) & 1u)) continue;
        bool first = true;
        for (int32_t z = b; z < e && first; ++z) {
            const ArcRec q = arcs[z];
            if (q.y == r.y && (q.w < r.w || (q.w == r.w && z < x))) first = false;
        }
        if (first) atomicAdd(&seed_hist[dist_bin(r.w)], 1u);
    }
}

__global__ __launch_bounds__(64) void k_kcp_seed_bound(const uint32_t *seed_hist, uint32_t k, QueryCtl *ctl) {
    const uint32_t b = wave_bound_from_hist(seed_hist, k);
    if (threadIdx.x == 0) ctl->theta = b;
}

// Keep the emitted pairs within the final bound (order is restored by the sort).
__global__ void k_kcp_filter(const rn_pair *pairs, unsigned long long cap, rn_pair *kept, QueryCtl *ctl) {
    const unsigned long long n = min(ctl->npairs, cap);
    const uint32_t bound = ctl->theta;
    for (unsigned long long i = blockIdx.x * static_cast<unsigned long long>(blockDim.x) + threadIdx.x;
         i < n; i += static_cast<unsigned long long>(gridDim.x) * blockDim.x) {
        const rn_pair p = pairs[i];
        if (p.dist <= bound) kept[atomicAdd(&ctl->nsel, 1ull)] = p;
    }
}

inline uint32_t bitlen(uint64_t x) {
    uint32_t b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

template <int HB>
hipError_t launch_join_tier(const JoinArgs &a, uint32_t max_sources, hipStream_t s) {
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
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_join<HB>, 64, 0);
        if (e != hipSuccess) return e;
        cus = prop.multiProcessorCount;
        resident = occ > 0 ? occ : 1;
    }
    uint64_t grid = static_cast<uint64_t>(cus) * resident;
    grid = (grid + 7) / 8 * 8;
    const uint64_t want = (static_cast<uint64_t>(max_sources) + 7) / 8 * 8;
    if (want < grid) grid = want;
    if (grid == 0) grid = 8;
    hipLaunchKernelGGL(k_join<HB>, dim3(static_cast<uint32_t>(grid)), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

size_t stage_scratch_words(int32_t V) {
    const size_t nwords = (static_cast<size_t>(V) + 31) / 32;
    return (nwords + 1023) / 1024 + 1;
}

hipError_t launch_stage(const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, int32_t V,
                        const int32_t *rank, const int32_t *order, uint32_t *rbits,
                        uint32_t *sbits, int32_t *src, QueryCtl *ctl, uint32_t *scratch,
                        hipStream_t s) {
    const int64_t n = static_cast<int64_t>(nR) + nS;
    hipLaunchKernelGGL(k_mark, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, s, R, nR, S,
                       nS, V, rank, rbits, sbits, ctl);
    hipLaunchKernelGGL(k_overlap, dim3(static_cast<uint32_t>((nR + 255) / 256)), dim3(256), 0, s, R, nR,
                       V, sbits, ctl);
    const uint32_t nwords = static_cast<uint32_t>((static_cast<int64_t>(V) + 31) / 32);
    const uint32_t nblk = (nwords + 1023u) / 1024u;
    hipLaunchKernelGGL(k_rank_count, dim3(nblk), dim3(1024), 0, s, rbits, nwords, scratch);
    hipLaunchKernelGGL(k_rank_emit, dim3(nblk), dim3(1024), 0, s, rbits, nwords, scratch, order, src, ctl);
    return hipGetLastError();
}

int join_tier_supported(int hash_log2) { return hash_log2 >= 8 && hash_log2 <= 14; }

hipError_t launch_join(const JoinArgs &a, int hash_log2, uint32_t max_sources, hipStream_t s) {
    switch (hash_log2) {
        case 8: return launch_join_tier<8>(a, max_sources, s);
        case 9: return launch_join_tier<9>(a, max_sources, s);
        case 10: return launch_join_tier<10>(a, max_sources, s);
        case 11: return launch_join_tier<11>(a, max_sources, s);
        case 12: return launch_join_tier<12>(a, max_sources, s);
        case 13: return launch_join_tier<13>(a, max_sources, s);
        case 14: return launch_join_tier<14>(a, max_sources, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_join_global(const JoinArgs &a, uint32_t *slots, uint32_t nslots, int32_t V,
                              uint32_t max_sources, hipStream_t s) {
    uint32_t grid = nslots < max_sources ? nslots : max_sources;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_join_global, dim3(grid), dim3(256), 0, s, a, slots, global_slot_words(V), V);
    return hipGetLastError();
}

// per pass: a [256 digits][kSortBlocks tiles] histogram, then 256 digit totals
size_t sort_hist_words() { return static_cast<size_t>(kSortPassesMax + 1) * 256u * (kSortBlocks + 1); }

hipError_t launch_sort_to_out(rn_pair *pairs, rn_pair *scratch, const unsigned long long *n,
                              unsigned long long cap, uint32_t max_dist, int32_t V, uint32_t *hist,
                              rn_pair *out, unsigned long long user_cap, unsigned long long out_limit,
                              const QueryCtl *ctl, int last_tier, hipStream_t s) {
    const uint32_t vb = V > 1 ? bitlen(static_cast<uint64_t>(V - 1)) : 1u;
    const uint32_t bits = 2u * vb + bitlen(max_dist);
    const uint32_t passes = (bits + 7u) / 8u;
    if (bits <= 64 && cap < (1ull << 31)) {
        uint64_t *ka = reinterpret_cast<uint64_t *>(scratch);
        uint64_t *kb = reinterpret_cast<uint64_t *>(pairs);   // records are packed into ka first
        const size_t hw = 256u * kSortBlocks;
        uint32_t *tot = hist + (kSortPassesMax + 1) * hw;
        hipLaunchKernelGGL(k_sort_pack, dim3(kSortBlocks), dim3(256), 0, s, pairs, ka, n, cap, vb, hist);
        uint64_t *in = ka, *o = kb;
        for (uint32_t p = 0; p < passes; ++p) {
            const bool last = p + 1 == passes;
            hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(256), 0, s, hist + p * hw, tot + p * 256u);
            hipLaunchKernelGGL(k_sort_pass, dim3(kSortBlocks), dim3(256), 0, s, in, o, last ? out : nullptr,
                               n, cap, 8u * p, vb, hist + p * hw, tot + p * 256u,
                               last ? nullptr : hist + (p + 1) * hw, 8u * (p + 1), ctl, user_cap, out_limit,
                               last_tier);
            uint64_t *t = in;
            in = o;
            o = t;
        }
        return hipGetLastError();
    }
    rn_pair *in = pairs, *o = scratch;
    uint32_t *tot = hist + 256u * kSortBlocks;
    for (uint32_t bit = 0; bit < bits; bit += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(kSortBlocks), dim3(256), 0, s, in, n, cap, bit, vb, hist);
        hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(256), 0, s, hist, tot);
        hipLaunchKernelGGL(k_radix_scatter, dim3(kSortBlocks), dim3(256), 0, s, in, o, n, cap, bit, vb,
                           hist, tot);
        rn_pair *t = in;
        in = o;
        o = t;
    }
    return launch_copy_out(in, out, n, ctl, user_cap, cap, out_limit, last_tier, s);
}

hipError_t launch_copy_out(const rn_pair *src, rn_pair *dst, const unsigned long long *n,
                           const QueryCtl *ctl, unsigned long long user_cap, unsigned long long limit,
                           unsigned long long out_limit, int last_tier, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_out, dim3(1024), dim3(256), 0, s, src, dst, n, ctl, user_cap, limit, out_limit,
                       last_tier);
    return hipGetLastError();
}

hipError_t launch_kcp_seed(const int32_t *src, const uint32_t *nsrc, uint32_t max_sources,
                           const int32_t *row_ptr, const ArcRec *arcs, const uint32_t *sbits,
                           uint32_t *seed_hist, uint32_t k, QueryCtl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_kcp_seed_hist, dim3((max_sources + 255) / 256), dim3(256), 0, s, src, nsrc, row_ptr,
                       arcs, sbits, seed_hist);
    hipLaunchKernelGGL(k_kcp_seed_bound, dim3(1), dim3(64), 0, s, seed_hist, k, ctl);
    return hipGetLastError();
}

hipError_t launch_kcp_filter(const rn_pair *pairs, unsigned long long cap, rn_pair *kept, QueryCtl *ctl,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_kcp_filter, dim3(1024), dim3(256), 0, s, pairs, cap, kept, ctl);
    return hipGetLastError();
}

}  // namespace rn
