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

constexpr uint32_t kEmpty = 0x7FFFFFFFu;  // empty table key (never a vertex id)
constexpr uint32_t kPend = 0x80000000u;   // key flag: the vertex is in the pending list
constexpr uint32_t kWin = 256;            // arcs expanded per window (4 per lane)

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint32_t popc(uint64_t m) { return static_cast<uint32_t>(__popcll(m)); }

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), o)));
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = static_cast<uint32_t>(__shfl_up(static_cast<int>(v), o));
        if (lane >= static_cast<uint32_t>(o)) v += t;
    }
    return v;
}

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
// PC bounds the pending set and the frontier of one bucket; the table holds
// every vertex reached within the bound.
template <int HB>
struct Tier {
    static constexpr int H = 1 << HB;
    static constexpr int PC = HB <= 9 ? 128 : (HB <= 11 ? 256 : (HB == 12 ? 512 : 1024));
    static constexpr int U = (H / 64) < 8 ? (H / 64) : 8;   // table rows scanned per batch
};

template <int HB>
struct SearchLds {
    static constexpr int H = Tier<HB>::H;
    static constexpr int PC = Tier<HB>::PC;
    uint32_t key[H];    // vertex id | kPend, or kEmpty
    uint32_t dist[H];   // tentative distance (kInf when empty)
    uint32_t pslot[PC]; // pending list: table slot, arc range
    int32_t pbeg[PC];
    int32_t pend[PC];
    int32_t fbeg[PC];   // frontier of the current phase: arc range and distance
    int32_t fend[PC];   //   (reused as the emission staging area at the end)
    uint32_t fd[PC];
    uint8_t own[kWin];  // window arc -> owning frontier lane
};

struct WaveState {
    uint32_t np;    // pending count
    uint32_t nins;  // table entries in use
    uint32_t imin;  // per-lane min of improved distances this phase
    bool ovf;       // the search outgrew this tier
};

// Relax one arc per lane (act lanes), then append newly pending vertices.
// Must be called by all 64 lanes; st.ovf is wave-uniform afterwards.
template <int HB>
__device__ __forceinline__ void relax_append(SearchLds<HB> &L, WaveState &st, bool act, int32_t y,
                                             uint32_t nd, int32_t yb, int32_t ye) {
    constexpr int H = Tier<HB>::H;
    constexpr int PC = Tier<HB>::PC;
    bool ins = false, app = false, lost = false;
    uint32_t h = 0;
    if (act) {
        h = slot_hash<HB>(static_cast<uint32_t>(y));
        bool found = false;
        for (int probe = 0; probe < H; ++probe) {
            uint32_t k = lds_load(&L.key[h]);
            if ((k & ~kPend) == static_cast<uint32_t>(y)) { found = true; break; }
            if (k == kEmpty) {
                uint32_t old = atomicCAS(&L.key[h], kEmpty, static_cast<uint32_t>(y));
                if (old == kEmpty) { ins = true; found = true; break; }
                if ((old & ~kPend) == static_cast<uint32_t>(y)) { found = true; break; }
            }
            h = (h + 1) & (H - 1);
        }
        if (found) {
            uint32_t old = atomicMin(&L.dist[h], nd);
            if (nd < old) {
                st.imin = min(st.imin, nd);
                uint32_t ko = atomicOr(&L.key[h], kPend);
                app = (ko & kPend) == 0;
            }
        } else {
            lost = true;
        }
    }
    const uint64_t mI = __ballot(ins), mA = __ballot(app), mL = __ballot(lost);
    st.nins += popc(mI);
    const uint32_t na = popc(mA);
    if (mL != 0 || st.nins > (3u * H) / 4u || st.np + na > static_cast<uint32_t>(PC)) {
        st.ovf = true;
        return;
    }
    if (app) {
        const uint32_t r = st.np + mbcnt(mA);
        L.pslot[r] = h;
        L.pbeg[r] = yb;
        L.pend[r] = ye;
    }
    st.np += na;
}

__device__ __forceinline__ uint32_t current_bound(const JoinArgs &a) {
    if (!a.kcp) return a.theta;
    uint32_t t = __hip_atomic_load(&a.ctl->theta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return min(t, a.theta);
}

// Write this wave's staged pairs (L.fbeg = v, L.fd = dist) for source u.
template <int HB>
__device__ __forceinline__ void flush_pairs(SearchLds<HB> &L, const JoinArgs &a, int32_t u,
                                            uint32_t &nst) {
    if (nst == 0) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&a.ctl->npairs, static_cast<unsigned long long>(nst));
    const uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(base & 0xFFFFFFFFull), 0));
    const uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(base >> 32), 0));
    base = (static_cast<unsigned long long>(hi) << 32) | lo;
    wave_sync();
    for (uint32_t i = lane_id(); i < nst; i += 64) {
        const unsigned long long idx = base + i;
        if (idx < a.pair_cap) {
            rn_pair p;
            p.u = u;
            p.v = L.fbeg[i];
            p.dist = L.fd[i];
            a.pairs[idx] = p;
        }
    }
    wave_sync();
    nst = 0;
}

// Bounded search from u.  Bucket b holds tentative distances in
// [b*delta, (b+1)*delta); each phase takes every pending vertex of the lowest
// non-empty bucket, expands its arcs and relaxes their targets.  With
// delta <= the smallest arc weight each vertex is expanded once, at its final
// distance (Dijkstra order by buckets); a larger delta trades re-expansions for
// fewer phases, and delta = 0 expands the whole pending set every phase.  The
// search ends when nothing is pending; every table entry then holds its exact
// distance, and entries in S become pairs.
template <int HB>
__device__ void search_source(SearchLds<HB> &L, const JoinArgs &a, int32_t u) {
    constexpr int H = Tier<HB>::H;
    constexpr int U = Tier<HB>::U;
    const uint32_t lane = lane_id();
    const int32_t ub = a.row_ptr[u];
    const int32_t ue = a.row_ptr[u + 1];
    if (lane == 0) {
        const uint32_t h0 = slot_hash<HB>(static_cast<uint32_t>(u));   // table is empty
        lds_store(&L.key[h0], static_cast<uint32_t>(u) | kPend);
        L.dist[h0] = 0;
        L.pslot[0] = h0;
        L.pbeg[0] = ub;
        L.pend[0] = ue;
    }
    wave_sync();
    WaveState st;
    st.np = 1;
    st.nins = 1;
    st.ovf = false;
    uint32_t pmin = 0;
    uint32_t bound = a.theta;

    while (st.np > 0) {
        bound = current_bound(a);
        uint32_t thr = kInf;
        if (a.delta != 0) {
            const uint64_t t = (static_cast<uint64_t>(pmin / a.delta) + 1ull) * a.delta;
            thr = t > kInf ? kInf : static_cast<uint32_t>(t);
        }
        // ---- split the pending list into this phase's frontier and the rest
        uint32_t nf = 0, nk = 0, kmin = kInf;
        for (uint32_t base = 0; base < st.np; base += 64) {
            const uint32_t i = base + lane;
            const bool valid = i < st.np;
            uint32_t s = 0, d = kInf;
            int32_t b = 0, e = 0;
            if (valid) {
                s = L.pslot[i];
                b = L.pbeg[i];
                e = L.pend[i];
                d = L.dist[s];
            }
            const bool isF = valid && d < thr && d <= bound;
            const bool isK = valid && d >= thr && d <= bound;
            const uint64_t mF = __ballot(isF), mK = __ballot(isK);
            wave_sync();  // every lane has read its entry before the in-place compaction
            if (valid && !isK) atomicAnd(&L.key[s], ~kPend);
            if (isF) {
                const uint32_t r = nf + mbcnt(mF);
                L.fbeg[r] = b;
                L.fend[r] = e;
                L.fd[r] = d;
            }
            if (isK) {
                const uint32_t r = nk + mbcnt(mK);
                L.pslot[r] = s;
                L.pbeg[r] = b;
                L.pend[r] = e;
                kmin = min(kmin, d);
            }
            nf += popc(mF);
            nk += popc(mK);
        }
        st.np = nk;
        st.imin = kInf;
        wave_sync();
        // ---- expand the frontier, kWin arcs at a time
        for (uint32_t fb = 0; fb < nf && !st.ovf; fb += 64) {
            const uint32_t f = fb + lane;
            int32_t b = 0, e = 0;
            uint32_t d = 0;
            if (f < nf) {
                b = L.fbeg[f];
                e = L.fend[f];
                d = L.fd[f];
            }
            const uint32_t deg = static_cast<uint32_t>(e - b);
            const uint32_t incl = wave_incl_scan(deg);
            const uint32_t excl = incl - deg;
            const uint32_t total = static_cast<uint32_t>(__shfl(static_cast<int>(incl), 63));
            for (uint32_t wb = 0; wb < total && !st.ovf; wb += kWin) {
                const uint32_t lo = max(excl, wb), hi = min(excl + deg, wb + kWin);
                for (uint32_t p = lo; p < hi; ++p) L.own[p - wb] = static_cast<uint8_t>(lane);
                wave_sync();
                const uint32_t cnt = min(kWin, total - wb);
                ArcRec r[kWin / 64];
                uint32_t nd[kWin / 64];
#pragma unroll
                for (int j = 0; j < static_cast<int>(kWin / 64); ++j) {
                    const uint32_t t = j * 64 + lane;
                    const bool act = t < cnt;
                    const uint32_t o = act ? L.own[t] : 0u;
                    const int32_t ob = __shfl(b, static_cast<int>(o));
                    const uint32_t ox = static_cast<uint32_t>(__shfl(static_cast<int>(excl), static_cast<int>(o)));
                    const uint32_t od = static_cast<uint32_t>(__shfl(static_cast<int>(d), static_cast<int>(o)));
                    nd[j] = kInf;
                    r[j].y = 0;
                    r[j].ybeg = 0;
                    r[j].yend = 0;
                    if (act) {
                        r[j] = a.arcs[ob + static_cast<int32_t>(wb + t - ox)];
                        nd[j] = sat_add(od, r[j].w);
                    }
                }
                wave_sync();  // own[] fully read before the next window rewrites it
#pragma unroll
                for (int j = 0; j < static_cast<int>(kWin / 64); ++j) {
                    relax_append<HB>(L, st, nd[j] <= bound, r[j].y, nd[j], r[j].ybeg, r[j].yend);
                    if (st.ovf) break;
                }
                wave_sync();
            }
        }
        pmin = min(wave_min(kmin), wave_min(st.imin));
        if (st.ovf) break;
    }

    // ---- emit table entries in S, and clear the table for the next source
    bound = current_bound(a);
    uint32_t nst = 0;
    unsigned long long warcs = 0;
    uint32_t wsettled = 0;
    for (uint32_t g0 = 0; g0 < static_cast<uint32_t>(H); g0 += 64 * U) {
        uint32_t k[U], d[U], sb[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t slot = g0 + j * 64 + lane;
            k[j] = lds_load(&L.key[slot]);
            d[j] = L.dist[slot];
            sb[j] = 0;
            if (!st.ovf && k[j] != kEmpty) sb[j] = a.sbits[(k[j] & ~kPend) >> 5];
        }
        if (a.count_work && !st.ovf) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                if (k[j] != kEmpty && d[j] <= bound) {
                    const uint32_t y = k[j] & ~kPend;
                    warcs += static_cast<unsigned long long>(a.row_ptr[y + 1] - a.row_ptr[y]);
                    wsettled += 1;
                }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t slot = g0 + j * 64 + lane;
            lds_store(&L.key[slot], kEmpty);
            L.dist[slot] = kInf;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t y = k[j] & ~kPend;
            const bool m = !st.ovf && k[j] != kEmpty && ((sb[j] >> (y & 31u)) & 1u) && d[j] <= bound;
            const uint64_t mM = __ballot(m);
            if (m) {
                const uint32_t r = nst + mbcnt(mM);
                L.fbeg[r] = static_cast<int32_t>(y);
                L.fd[r] = d[j];
            }
            nst += popc(mM);
            if (nst + 64 > static_cast<uint32_t>(Tier<HB>::PC)) {
                wave_sync();
                flush_pairs<HB>(L, a, u, nst);
            }
        }
    }
    wave_sync();
    flush_pairs<HB>(L, a, u, nst);
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
        L.dist[i] = kInf;
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

// List the marked ranks in increasing order as vertex ids (one block).
__global__ __launch_bounds__(1024) void k_compact(const uint32_t *rbits, uint32_t nwords,
                                                  const int32_t *order, int32_t *src,
                                                  QueryCtl *ctl) {
    __shared__ uint32_t wsum[16];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (nwords + 1023u) / 1024u;
    const uint32_t beg = min(nwords, tid * per), end = min(nwords, beg + per);
    uint32_t c = 0;
    for (uint32_t w = beg; w < end; ++w) c += __popc(rbits[w]);
    const uint32_t incl = wave_incl_scan(c);
    if ((tid & 63u) == 63u) wsum[tid >> 6] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < (tid >> 6); ++w) off += wsum[w];
    uint32_t pos = off + incl - c;
    for (uint32_t w = beg; w < end; ++w) {
        uint32_t bits = rbits[w];
        while (bits) {
            const uint32_t b = __ffs(bits) - 1u;
            const int32_t r = static_cast<int32_t>(w * 32u + b);
            src[pos++] = order ? order[r] : r;
            bits &= bits - 1u;
        }
    }
    if (tid == 1023u) ctl->nsrc = pos;
}

// ------------------------------------------------------------------ radix sort
constexpr uint32_t kSortBlocks = 256;

// 8-bit digit at `bit` of the key (dist, u, v) packed as dist:u:v with vb bits per id.
__device__ __forceinline__ uint32_t pair_digit(const rn_pair &p, uint32_t bit, uint32_t vb) {
    const uint32_t sh = 2u * vb;
    if (bit >= sh) return (p.dist >> (bit - sh)) & 255u;
    const uint64_t lo = (static_cast<uint64_t>(static_cast<uint32_t>(p.u)) << vb) |
                        static_cast<uint32_t>(p.v);
    uint64_t x = lo >> bit;
    if (bit + 8u > sh) x |= static_cast<uint64_t>(p.dist) << (sh - bit);
    return static_cast<uint32_t>(x) & 255u;
}

__device__ __forceinline__ void sort_tile(const unsigned long long *nptr, unsigned long long cap,
                                          uint64_t &beg, uint64_t &end) {
    const uint64_t n = min(static_cast<uint64_t>(*nptr), static_cast<uint64_t>(cap));
    const uint64_t tile = (n + gridDim.x - 1) / gridDim.x;
    beg = min(n, blockIdx.x * tile);
    end = min(n, beg + tile);
}

__global__ __launch_bounds__(256) void k_radix_hist(const rn_pair *in, const unsigned long long *nptr,
                                                    unsigned long long cap, uint32_t bit,
                                                    uint32_t vb, uint32_t *hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t beg, end;
    sort_tile(nptr, cap, beg, end);
    for (uint64_t i = beg + threadIdx.x; i < end; i += 256) atomicAdd(&h[pair_digit(in[i], bit, vb)], 1u);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of hist[256 * kSortBlocks] in place (one block).
__global__ __launch_bounds__(1024) void k_radix_scan(uint32_t *hist) {
    __shared__ uint32_t wsum[16];
    constexpr uint32_t per = 256u * kSortBlocks / 1024u;
    const uint32_t tid = threadIdx.x;
    uint32_t c = 0;
    for (uint32_t i = 0; i < per; ++i) c += hist[tid * per + i];
    const uint32_t incl = wave_incl_scan(c);
    if ((tid & 63u) == 63u) wsum[tid >> 6] = incl;
    __syncthreads();
    uint32_t run = incl - c;
    for (uint32_t w = 0; w < (tid >> 6); ++w) run += wsum[w];
    for (uint32_t i = 0; i < per; ++i) {
        const uint32_t v = hist[tid * per + i];
        hist[tid * per + i] = run;
        run += v;
    }
}

// Stable scatter by digit: items keep their input order within a digit.
__global__ __launch_bounds__(256) void k_radix_scatter(const rn_pair *in, rn_pair *out,
                                                       const unsigned long long *nptr,
                                                       unsigned long long cap, uint32_t bit,
                                                       uint32_t vb, const uint32_t *hist) {
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[4][256];
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    base[tid] = hist[tid * gridDim.x + blockIdx.x];
    uint64_t beg, end;
    sort_tile(nptr, cap, beg, end);
    for (uint64_t c = beg; c < end; c += 256) {
#pragma unroll
        for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const uint64_t i = c + tid;
        const bool act = i < end;
        rn_pair p{0, 0, 0};
        uint32_t dg = 0;
        if (act) {
            p = in[i];
            dg = pair_digit(p, bit, vb);
        }
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
        if (act) {
            uint32_t off = 0;
            for (uint32_t w = 0; w < wave; ++w) off += wcnt[w][dg];
            out[base[dg] + off + wrank] = p;
        }
        __syncthreads();
        base[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

__global__ void k_copy_out(const rn_pair *src, rn_pair *dst, const QueryCtl *ctl,
                           unsigned long long user_cap, unsigned long long limit, int last_tier) {
    const unsigned long long n = ctl->npairs;
    if (ctl->err != 0 || n > user_cap || n > limit) return;
    if (last_tier >= 0 && ctl->novf[last_tier] != 0) return;
    for (unsigned long long i = blockIdx.x * static_cast<unsigned long long>(blockDim.x) + threadIdx.x;
         i < n; i += static_cast<unsigned long long>(gridDim.x) * blockDim.x)
        dst[i] = src[i];
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

hipError_t launch_stage(const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, int32_t V,
                        const int32_t *rank, const int32_t *order, uint32_t *rbits,
                        uint32_t *sbits, int32_t *src, QueryCtl *ctl, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(nR) + nS;
    hipLaunchKernelGGL(k_mark, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, s, R, nR, S,
                       nS, V, rank, rbits, sbits, ctl);
    hipLaunchKernelGGL(k_overlap, dim3(static_cast<uint32_t>((nR + 255) / 256)), dim3(256), 0, s, R, nR,
                       V, sbits, ctl);
    const uint32_t nwords = static_cast<uint32_t>((static_cast<int64_t>(V) + 31) / 32);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, rbits, nwords, order, src, ctl);
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

size_t sort_hist_words() { return 256u * kSortBlocks; }

hipError_t launch_sort_pairs(rn_pair *a, rn_pair *b, const unsigned long long *n,
                             unsigned long long cap, uint32_t max_dist, int32_t V, uint32_t *hist,
                             rn_pair **out_buf, hipStream_t s) {
    const uint32_t vb = V > 1 ? bitlen(static_cast<uint64_t>(V - 1)) : 1u;
    const uint32_t bits = 2u * vb + bitlen(max_dist);
    rn_pair *in = a, *out = b;
    for (uint32_t bit = 0; bit < bits; bit += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(kSortBlocks), dim3(256), 0, s, in, n, cap, bit, vb, hist);
        hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, s, hist);
        hipLaunchKernelGGL(k_radix_scatter, dim3(kSortBlocks), dim3(256), 0, s, in, out, n, cap, bit,
                           vb, hist);
        rn_pair *t = in;
        in = out;
        out = t;
    }
    *out_buf = in;
    return hipGetLastError();
}

hipError_t launch_copy_out(const rn_pair *src, rn_pair *dst, const QueryCtl *ctl,
                           unsigned long long user_cap, unsigned long long limit, int last_tier,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_copy_out, dim3(1024), dim3(256), 0, s, src, dst, ctl, user_cap, limit,
                       last_tier);
    return hipGetLastError();
}

}  // namespace rn
