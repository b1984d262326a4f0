// rn_noalloc.cpp -- rn_dist_join_noalloc: the theta-join with every device
// buffer of the call carved from one file-scope device array, for callers
// that cannot allocate device memory (include/rn.h).
//
// The launch sequence is the one of rn_dist_join (stage, relax, sort); only
// the buffers differ: the call block, descriptors, staging scratch, source
// and re-run lists, record buffers, the call-state copy and (when a search
// needs it) global-tier slots all live in `scratch`, whose device address is
// taken once per device with hipGetSymbolAddress.  Calls on one device share
// the array, so calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "rn.h"
#include "rn_host.h"
#include "rn_internal.h"

using namespace rn;
using namespace rn::host;

// The scratch array (RN_NOALLOC_SCRATCH_BYTES per device).  In host code its
// name stands for a host-side shadow, so it is only ever reached through the
// device address kept in g_scratch.
static __device__ __align__(256) uint32_t scratch[size_t{RN_NOALLOC_SCRATCH_BYTES} / 4];

namespace {

constexpr size_t kScratchWords = size_t{RN_NOALLOC_SCRATCH_BYTES} / 4;
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
uint32_t *g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device (taken once per device).
rn_status scratch_ptr(int dev, uint32_t **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(RN_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "locating the scratch array");
        g_scratch[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch[dev];
    return RN_OK;
}

// Carve a workspace for prepared call p out of the scratch words [base,
// base + kScratchWords); nslots global-tier slots for graphs of Vmax vertices
// (0: none).  The record buffers take what is left.  Returns RN_ERR_NOMEM if
// the fixed part does not fit.
rn_status carve(uint32_t *base, const Prepared &p, int32_t Vmax, uint32_t nslots, Workspace &ws, size_t *slot_words) {
    size_t at = 0;
    auto take = [&](size_t words) {
        uint32_t *q = base + at;
        at = round_up(at + words, 64);   // 256-byte aligned regions
        return q;
    };
    ws = Workspace{};
    const size_t state_words = (sizeof(CallCtl) + static_cast<size_t>(p.nq) * sizeof(QueryState)) / 4;
    const size_t nsrc = std::max<size_t>(p.total_R, 1);
    const size_t fixed = round_up(p.block_words, 64) + round_up((p.desc_bytes + 3) / 4, 64) +
                         round_up(stage_scratch_words(p.rbits_words), 64) + round_up(state_words, 64) +
                         (2 + 2 * kLists) * round_up(nsrc, 64);
    const size_t sw = nslots ? global_slot_words(Vmax) : 0;
    if (fixed + nslots * sw + 64 * 8 > kScratchWords) return fail(RN_ERR_NOMEM, "the call does not fit the scratch array");
    ws.d_block = take(p.block_words);
    ws.block_words = p.block_words;
    ws.d_desc = reinterpret_cast<uint8_t *>(take((p.desc_bytes + 3) / 4));
    ws.desc_bytes = p.desc_bytes;
    ws.d_stage = take(stage_scratch_words(p.rbits_words));
    ws.stage_words = stage_scratch_words(p.rbits_words);
    ws.d_state_map = take(state_words);
    ws.d_src = reinterpret_cast<int32_t *>(take(nsrc));
    ws.d_srcq = take(nsrc);
    for (int i = 0; i < kLists; ++i) {
        ws.d_list[i] = reinterpret_cast<int32_t *>(take(nsrc));
        ws.d_listq[i] = take(nsrc);
    }
    ws.src_cap = nsrc;
    if (nslots) {
        ws.d_gslots = take(nslots * sw);
        ws.n_gslots = nslots;
    }
    *slot_words = sw;
    const size_t left = kScratchWords - at;
    if (left < 8 * 4096) return fail(RN_ERR_NOMEM, "the call does not fit the scratch array");
    const unsigned long long rec_cap = std::min<unsigned long long>(left / 8 - 16, kRecCapMax - 1);
    ws.d_recs[0] = reinterpret_cast<Rec *>(take(rec_cap * 4));
    ws.d_recs[1] = reinterpret_cast<Rec *>(take(rec_cap * 4));
    ws.rec_cap = rec_cap;
    return RN_OK;
}

}  // namespace

extern "C" {

rn_status rn_dist_join_noalloc(rn_graph *g, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS,
                               uint32_t theta, rn_pair *out, int64_t cap, int64_t *n_out, void *stream) {
    if (!n_out) return fail(RN_ERR_ARG, "n_out is NULL");
    *n_out = 0;
    if (!g) return fail(RN_ERR_ARG, "graph handle is NULL");
    if (cap < 0 || (cap > 0 && !out)) return fail(RN_ERR_ARG, "bad output buffer");
    rn_query q;
    std::memset(&q, 0, sizeof(q));
    q.R = R;
    q.S = S;
    q.nR = nR;
    q.nS = nS;
    q.theta = theta;
    q.delta = RN_DELTA_DEFAULT;
    RN_TRY(check_queries(g, &q, 1, nullptr));
    BusyGuard guard(g);
    if (!guard.ok) return fail(RN_ERR_BUSY, "handle in use by another call");
    RN_HIP(hipSetDevice(g->device), "selecting the device");
    uint32_t *base = nullptr;
    RN_TRY(scratch_ptr(g->device, &base));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // host-side plan of the call: kept per thread, so that after a thread's
    // first call its vectors are reused in place
    static thread_local Prepared p;
    RN_TRY(prepare(g, &q, 1, p));
    alignas(16) uint8_t h_desc[512];
    if (p.desc_bytes > sizeof(h_desc)) return fail(RN_ERR_DEVICE, "query descriptors too large");
    const size_t state_bytes = sizeof(CallCtl) + sizeof(QueryState);
    alignas(16) uint8_t h_state[sizeof(CallCtl) + sizeof(QueryState)];
    uint32_t nslots = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        Workspace ws;
        size_t slot_words = 0;
        RN_TRY(carve(base, p, g->Vmax, nslots, ws, &slot_words));
        if (nslots) {
            // global-tier slots start cleared (every word all ones; the layout
            // depends on the graph, so clear at every use)
            RN_HIP(launch_fill_u32(ws.d_gslots, global_clear_words(nslots, g->Vmax), 0xFFFFFFFFu, s),
                   "clearing search slots");
        }
        fill_host_desc(p, h_desc);
        RN_HIP(hipMemcpyAsync(ws.d_desc, h_desc, p.desc_bytes, hipMemcpyHostToDevice, s), "uploading the query");
        RN_TRY(enqueue_call(g, ws, p, out, cap, s, false));
        RN_HIP(hipMemcpyAsync(h_state, ws.d_state_map, state_bytes, hipMemcpyDeviceToHost, s), "reading the call state");
        RN_HIP(hipStreamSynchronize(s), "waiting for the call");
        CallCtl c;
        QueryState qs;
        std::memcpy(&c, h_state, sizeof(c));
        std::memcpy(&qs, h_state + sizeof(CallCtl), sizeof(qs));
        if (c.nlist[2] > 0 && nslots == 0) {
            // some search outgrew every on-chip table: run again with as many
            // global-tier slots as fit beside the other buffers (at most 8)
            const size_t sw = global_slot_words(g->Vmax);
            const size_t fixed = kScratchWords / 2;
            nslots = static_cast<uint32_t>(std::min<size_t>(8, fixed / std::max<size_t>(sw, 1)));
            if (nslots == 0)
                return fail(RN_ERR_NOMEM, "a search needs the global tier, whose slots do not fit the scratch array");
            continue;
        }
        if (c.npairs > ws.rec_cap)
            return fail(RN_ERR_NOMEM, "the call's records do not fit the scratch array (" + std::to_string(c.npairs) +
                                          " records, room for " + std::to_string(ws.rec_cap) + ")");
        if (c.resort) {   // the call's sort left the output to the radix sort
            RN_TRY(enqueue_sort_fallback(ws, p, out, cap, s));
            RN_HIP(hipStreamSynchronize(s), "waiting for the sort");
        }
        *n_out = static_cast<int64_t>(c.nout);
        if (qs.err) return fail(RN_ERR_ARG, "invalid node sets:" + describe_err(qs.err));
        if (c.nout > static_cast<unsigned long long>(cap)) return fail(RN_ERR_CAPACITY, "output buffer too small");
        return RN_OK;
    }
    return fail(RN_ERR_NOMEM, "the call did not settle");
}

}  // extern "C"
