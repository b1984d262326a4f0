// rn_server.cpp -- the request server: continuous batching of joins on a
// resident graph (include/rn.h, rn_server_*).
//
// One host thread owns the device work.  Submitted requests wait in a FIFO
// queue; whenever one of the server's lanes is free, the thread admits the
// longest prefix of the queue that fits the memory budget (estimated device
// footprint of each request) and the batch limit, and launches it on that
// lane as one batched call (rn_join_batch's launch sequence).  Lanes run on
// their own streams with their own buffers and global-tier slots, so a batch
// admitted while others are still on the device overlaps with them.  A lane
// is polled through events; its results are copied back without blocking the
// loop, and a batch whose records or output outgrow the lane's buffers is
// re-run with larger ones (results never depend on batching).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rn.h"
#include "rn_host.h"
#include "rn_internal.h"

using namespace rn;
using namespace rn::host;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
    int64_t id = 0;
    std::vector<int32_t> R, S;
    uint32_t theta = 0;
    int32_t k = 0;
    double footprint = 0;           // estimated device bytes while in flight
    bool heavy = false;             // estimated search work above kHeavyWork
    bool held = false;              // was once held back by the HBM budget
    Clock::time_point t_submit, t_done;
    std::vector<rn_pair> result;
    rn_status status = RN_OK;
    std::string err;
    bool done = false;
};

struct Lane {
    Workspace ws;
    hipStream_t stream = nullptr;
    hipEvent_t ev_state = nullptr;  // the call and its status read-back finished
    hipEvent_t ev_copy = nullptr;   // the results are on the host
    int32_t *d_ids = nullptr;       // R and S of the batch's requests
    int32_t *h_ids = nullptr;
    size_t ids_cap = 0;
    rn_pair *d_out = nullptr;
    size_t out_cap = 0;
    rn_pair *h_out = nullptr;
    size_t h_out_cap = 0;
    std::vector<Request *> batch;
    std::vector<rn_query> q;
    Prepared prep;
    enum State { IDLE, RUNNING, COPYING } state = IDLE;
    double reserved = 0;
    unsigned long long nout = 0;
    int reruns = 0;

    void release() {
        ws.release();
        dev_free(d_ids);
        host_free(h_ids);
        dev_free(d_out);
        host_free(h_out);
        ids_cap = out_cap = h_out_cap = 0;
        if (ev_state) (void)hipEventDestroy(ev_state), ev_state = nullptr;
        if (ev_copy) (void)hipEventDestroy(ev_copy), ev_copy = nullptr;
        if (stream) (void)hipStreamDestroy(stream), stream = nullptr;
    }
    // every device buffer of the lane, the global-tier slots included
    size_t device_bytes(int32_t Vmax) const {
        return ws.block_words * 4 + ws.desc_bytes + ws.stage_words * 4 + ws.src_cap * 8 * (1 + kLists) +
               static_cast<size_t>(ws.rec_cap) * 2 * sizeof(Rec) + ids_cap * 4 + out_cap * sizeof(rn_pair) +
               gslot_bytes(ws, Vmax);
    }
};

}  // namespace

struct rn_server {
    rn_graph *g = nullptr;
    BusyGuard *guard = nullptr;
    rn_server_config cfg{};
    int32_t V = 0;                  // vertices of the served graph
    std::vector<Lane> lanes;
    std::thread thr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::unordered_map<int64_t, Request *> reqs;
    int64_t next_id = 1;
    bool stop = false;
    double budget_used = 0;
    double c_ball = 0;              // estimated fraction of the graph within theta, per theta^2
    rn_server_stats stats{};
    int in_flight_requests = 0;
};

namespace {

// Estimated device bytes of a request while it is in flight: its ids, two
// record buffers and the output for the pairs it is expected to produce.
double footprint(const rn_server *s, const Request &r) {
    const double nR = static_cast<double>(r.R.size()), nS = static_cast<double>(r.S.size());
    double pairs;
    if (r.k == 0) {
        const double th = static_cast<double>(r.theta);
        pairs = nR * nS * std::min(1.0, s->c_ball * th * th / std::max(1, s->V));
    } else {
        pairs = std::min(nR * nS, 4.0 * r.k + nR);
    }
    return 4.0 * (nR + nS) + pairs * (2.0 * sizeof(Rec) + sizeof(rn_pair));
}

// Estimated search work of a request, in vertices visited: its searches run
// from the smaller side; a theta-join's balls hold about c_ball theta^2
// vertices; a k-closest-pairs search reaches the ball holding about k of the
// |R| |S| pairs (the whole graph when k is a large share of them).
double work_estimate(const rn_server *s, const Request &r) {
    const double nR = static_cast<double>(r.R.size()), nS = static_cast<double>(r.S.size());
    const double V = static_cast<double>(std::max(1, s->V));
    double ball;
    if (r.k == 0) {
        const double th = static_cast<double>(r.theta);
        ball = std::min(V, s->c_ball * th * th);
    } else {
        ball = std::min(V, std::max(64.0, 4.0 * static_cast<double>(r.k) * V / (nR * nS)));
        if (r.theta < kMaxDist) ball = std::min(ball, s->c_ball * double(r.theta) * r.theta);
    }
    return std::min(nR, nS) * ball;
}

// Requests above this estimated work (vertices visited; about 2-5 ms of
// device time on road graphs) are heavy: with heavy_lane set they run one at
// a time on the last lane, so that light requests never queue behind them.
constexpr double kHeavyWork = 2.0e7;

void finish_request(rn_server *s, Request *r, rn_status st, const std::string &msg) {
    r->status = st;
    r->err = msg;
    r->t_done = Clock::now();
    r->done = true;
}

// Everything in a lane's batch fails with st (device errors).
void fail_batch(rn_server *s, Lane &L, rn_status st, const std::string &msg) {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Request *r : L.batch) finish_request(s, r, st, msg);
    s->budget_used -= L.reserved;
    s->in_flight_requests -= static_cast<int>(L.batch.size());
    L.batch.clear();
    L.reserved = 0;
    L.state = Lane::IDLE;
    s->cv_done.notify_all();
}

rn_status enqueue_lane(rn_server *s, Lane &L) {
    // the device is shared with the other lanes: one stream per lane (side
    // streams would share the few hardware queues with other lanes and
    // serialise their kernels) and one block per source, so that the blocks
    // of a long batch do not hold every CU until it ends
    // (the call's last kernel writes its state into the lane's mapped read-back buffer)
    RN_TRY(enqueue_call(s->g, L.ws, L.prep, L.d_out, static_cast<int64_t>(L.out_cap), L.stream, false, true));
    RN_HIP(hipEventRecord(L.ev_state, L.stream), "recording an event");
    L.state = Lane::RUNNING;
    return RN_OK;
}

// Upload a formed batch and launch it on lane L.
rn_status launch_lane(rn_server *s, Lane &L) {
    size_t words = 0;
    for (const Request *r : L.batch) words += r->R.size() + r->S.size();
    if (L.ids_cap < words) {
        dev_free(L.d_ids);
        host_free(L.h_ids);
        L.ids_cap = 0;
        const size_t cap = words + words / 4 + 4096;
        RN_HIP(dev_alloc(&L.d_ids, cap), "allocating request ids");
        RN_HIP(hipHostMalloc(reinterpret_cast<void **>(&L.h_ids), cap * sizeof(int32_t), 0), "allocating request ids");
        L.ids_cap = cap;
    }
    L.q.assign(L.batch.size(), rn_query{});
    size_t off = 0;
    for (size_t i = 0; i < L.batch.size(); ++i) {
        const Request *r = L.batch[i];
        std::memcpy(L.h_ids + off, r->R.data(), r->R.size() * sizeof(int32_t));
        std::memcpy(L.h_ids + off + r->R.size(), r->S.data(), r->S.size() * sizeof(int32_t));
        rn_query &q = L.q[i];
        q.R = L.d_ids + off;
        q.S = L.d_ids + off + r->R.size();
        q.nR = static_cast<int32_t>(r->R.size());
        q.nS = static_cast<int32_t>(r->S.size());
        q.graph = s->cfg.graph;
        q.k = r->k;
        q.theta = r->theta;
        q.delta = RN_DELTA_DEFAULT;
        q.hash_log2 = 0;
        off += r->R.size() + r->S.size();
    }
    RN_HIP(hipMemcpyAsync(L.d_ids, L.h_ids, words * sizeof(int32_t), hipMemcpyHostToDevice, L.stream),
           "uploading request ids");
    RN_TRY(prepare(s->g, L.q.data(), static_cast<int32_t>(L.q.size()), L.prep));
    RN_TRY(ensure_buffers(L.ws, L.prep));
    if (L.out_cap == 0) {
        L.out_cap = 1u << 16;
        RN_HIP(dev_alloc(&L.d_out, L.out_cap), "allocating the output");
    }
    fill_host_desc(L.prep, L.ws.h_desc);
    RN_HIP(hipMemcpyAsync(L.ws.d_desc, L.ws.h_desc, L.prep.desc_bytes, hipMemcpyHostToDevice, L.stream),
           "uploading queries");
    L.reruns = 0;
    return enqueue_lane(s, L);
}

// Move lane L forward if its device work has finished.  Returns true if it did.
bool progress_lane(rn_server *s, Lane &L) {
    if (L.state == Lane::RUNNING) {
        const hipError_t e = hipEventQuery(L.ev_state);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) {
            fail_batch(s, L, RN_ERR_DEVICE, std::string("device error: ") + hipGetErrorString(e));
            return true;
        }
        const CallCtl c = *reinterpret_cast<const CallCtl *>(L.ws.h_state);
        rn_status st = RN_OK;
        bool rerun = false;
        if (c.nlist[2] > 0 && !L.ws.d_gslots) {
            // a search needed the global tier, whose slots this lane allocates on first need
            st = ensure_gslots(L.ws, s->g->Vmax, c.nlist[2], L.stream);
            rerun = true;
        } else if (c.npairs > L.ws.rec_cap) {
            st = grow_recs(L.ws, c.npairs);
            rerun = true;
        } else if (c.nout > L.out_cap) {
            dev_free(L.d_out);
            L.out_cap = 0;
            const size_t cap = static_cast<size_t>(c.nout + c.nout / 4 + 1024);
            if (dev_alloc(&L.d_out, cap) != hipSuccess) st = fail(RN_ERR_NOMEM, "allocating the output");
            else L.out_cap = cap;
            rerun = true;
        }
        if (rerun && st == RN_OK && ++L.reruns <= 3) {
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->stats.reruns += 1;
            }
            st = enqueue_lane(s, L);
            if (st == RN_OK) return true;
        }
        if (rerun || st != RN_OK) {
            fail_batch(s, L, st == RN_OK ? RN_ERR_NOMEM : st, st == RN_OK ? "buffers did not settle" : last_error());
            return true;
        }
        if (c.resort) {
            // the call's sort left the output to the radix sort, which
            // writes it before the copy below on the same stream
            st = enqueue_sort_fallback(L.ws, L.prep, L.d_out, static_cast<int64_t>(L.out_cap), L.stream);
            if (st != RN_OK) {
                fail_batch(s, L, st, last_error());
                return true;
            }
        }
        L.nout = c.nout;
        if (L.h_out_cap < L.nout) {
            host_free(L.h_out);
            L.h_out_cap = 0;
            const size_t cap = static_cast<size_t>(L.nout + L.nout / 4 + 1024);
            if (hipHostMalloc(reinterpret_cast<void **>(&L.h_out), cap * sizeof(rn_pair), 0) != hipSuccess) {
                fail_batch(s, L, RN_ERR_NOMEM, "allocating the host output");
                return true;
            }
            L.h_out_cap = cap;
        }
        hipError_t e2 = hipSuccess;
        if (L.nout) e2 = hipMemcpyAsync(L.h_out, L.d_out, L.nout * sizeof(rn_pair), hipMemcpyDeviceToHost, L.stream);
        if (e2 == hipSuccess) e2 = hipEventRecord(L.ev_copy, L.stream);
        if (e2 != hipSuccess) {
            fail_batch(s, L, RN_ERR_DEVICE, std::string("copying results: ") + hipGetErrorString(e2));
            return true;
        }
        L.state = Lane::COPYING;
        return true;
    }
    if (L.state == Lane::COPYING) {
        const hipError_t e = hipEventQuery(L.ev_copy);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) {
            fail_batch(s, L, RN_ERR_DEVICE, std::string("device error: ") + hipGetErrorString(e));
            return true;
        }
        const QueryState *qs = reinterpret_cast<const QueryState *>(L.ws.h_state + sizeof(CallCtl));
        for (size_t i = 0; i < L.batch.size(); ++i) {
            Request *r = L.batch[i];
            r->result.assign(L.h_out + qs[i].off, L.h_out + qs[i].off + qs[i].nout);
        }
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t i = 0; i < L.batch.size(); ++i) {
            const Request *r = L.batch[i];
            if (r->k == 0 && qs[i].err == 0 && r->theta > 0 && r->theta < kMaxDist) {
                // learn the ball-size estimate from what theta-joins really
                // produced (read by rn_server_submit under the same lock)
                const double c = static_cast<double>(qs[i].npairs) * s->V /
                                 (static_cast<double>(r->R.size()) * r->S.size() * double(r->theta) * r->theta);
                s->c_ball = 0.8 * s->c_ball + 0.2 * c;
            }
        }
        for (size_t i = 0; i < L.batch.size(); ++i) {
            Request *r = L.batch[i];
            if (qs[i].err) finish_request(s, r, RN_ERR_ARG, "invalid node sets:" + describe_err(qs[i].err));
            else finish_request(s, r, RN_OK, std::string());
        }
        s->stats.completed += static_cast<int64_t>(L.batch.size());
        s->budget_used -= L.reserved;
        s->in_flight_requests -= static_cast<int>(L.batch.size());
        L.batch.clear();
        L.reserved = 0;
        L.state = Lane::IDLE;
        s->cv_done.notify_all();
        return true;
    }
    return false;
}

void server_loop(rn_server *s) {
    (void)hipSetDevice(s->g->device);
    while (true) {
        bool moved = false;
        for (Lane &L : s->lanes) moved |= progress_lane(s, L);
        std::vector<Lane *> to_launch;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            const int32_t nl = static_cast<int32_t>(s->lanes.size());
            const bool split = s->cfg.heavy_lane && nl >= 2;
            for (int32_t li = 0; li < nl; ++li) {
                Lane &L = s->lanes[static_cast<size_t>(li)];
                if (L.state != Lane::IDLE || !L.batch.empty() || s->pending.empty()) continue;
                // admit waiting requests in arrival order, within the budget and
                // the batch limit (one request always goes when nothing is in
                // flight).  heavy_lane: the last lane takes heavy requests, one
                // per batch, first, and light ones when no heavy one waits; the
                // other lanes take light requests, and the first heavy one
                // while the heavy lane is busy and no light request waits
                const bool alone = s->in_flight_requests == 0;
                const bool heavy_lane = split && li == nl - 1;
                const bool heavy_busy = split && s->lanes[static_cast<size_t>(nl - 1)].state != Lane::IDLE;
                auto take_first_heavy = [&]() {
                    for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
                        Request *r = *it;
                        if (!r->heavy) continue;
                        const bool fits = s->budget_used + r->footprint <= static_cast<double>(s->cfg.hbm_budget);
                        if (!fits && !alone && !r->held) {
                            r->held = true;
                            s->stats.budget_waits += 1;
                        }
                        if (!fits && !alone) return false;
                        s->pending.erase(it);
                        L.batch.push_back(r);
                        L.reserved += r->footprint;
                        s->budget_used += r->footprint;
                        s->in_flight_requests += 1;
                        return true;   // heavy requests go in arrival order, one per batch
                    }
                    return false;
                };
                bool took_heavy = heavy_lane && take_first_heavy();
                for (auto it = s->pending.begin();
                     !took_heavy && it != s->pending.end() && static_cast<int32_t>(L.batch.size()) < s->cfg.max_batch;) {
                    Request *r = *it;
                    if (split && r->heavy) {   // left for the heavy lane
                        ++it;
                        continue;
                    }
                    const bool fits = s->budget_used + r->footprint <= static_cast<double>(s->cfg.hbm_budget);
                    if (!fits && !(alone && L.batch.empty())) {
                        if (!r->held) {
                            r->held = true;
                            s->stats.budget_waits += 1;
                        }
                        break;
                    }
                    it = s->pending.erase(it);
                    L.batch.push_back(r);
                    L.reserved += r->footprint;
                    s->budget_used += r->footprint;
                    s->in_flight_requests += 1;
                }
                if (L.batch.empty() && split && !heavy_lane && heavy_busy) take_first_heavy();
                if (L.batch.empty()) continue;   // nothing this lane may take now
                to_launch.push_back(&L);
                s->stats.batches += 1;
                s->stats.peak_budget = std::max(s->stats.peak_budget, static_cast<int64_t>(s->budget_used));
                s->stats.max_batch_seen = std::max<int32_t>(s->stats.max_batch_seen, static_cast<int32_t>(L.batch.size()));
            }
            int busy = static_cast<int>(to_launch.size());
            for (const Lane &L : s->lanes) busy += L.state != Lane::IDLE ? 1 : 0;
            s->stats.max_lanes_busy = std::max<int32_t>(s->stats.max_lanes_busy, busy);
            s->stats.max_in_flight = std::max<int32_t>(s->stats.max_in_flight, s->in_flight_requests);
            if (to_launch.empty() && !moved) {
                bool idle = true;
                for (const Lane &L : s->lanes) idle &= L.state == Lane::IDLE;
                if (idle && s->pending.empty()) {
                    if (s->stop) break;
                    s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
                    continue;
                }
            }
        }
        for (Lane *L : to_launch) {
            const rn_status st = launch_lane(s, *L);
            if (st != RN_OK) fail_batch(s, *L, st, last_error());
        }
        if (!to_launch.empty() || moved) {
            size_t bytes = 0;
            for (const Lane &L : s->lanes) bytes += L.device_bytes(s->g->Vmax);
            std::lock_guard<std::mutex> lk(s->mu);
            s->stats.device_bytes = std::max<int64_t>(s->stats.device_bytes, static_cast<int64_t>(bytes));
        }
        if (to_launch.empty() && !moved) std::this_thread::yield();
    }
}

}  // namespace

extern "C" {

rn_status rn_server_create(rn_graph *g, const rn_server_config *cfg, rn_server **out) {
    if (!out) return fail(RN_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!g || !cfg) return fail(RN_ERR_ARG, "NULL argument");
    if (cfg->graph < 0 || cfg->graph >= g->ngraphs) return fail(RN_ERR_ARG, "graph index out of range");
    if (cfg->lanes < 1 || cfg->lanes > 16) return fail(RN_ERR_ARG, "lanes must be in [1, 16]");
    if (cfg->max_batch < 1 || cfg->max_batch > 65536) return fail(RN_ERR_ARG, "max_batch must be in [1, 65536]");
    if (cfg->hbm_budget < 1) return fail(RN_ERR_ARG, "hbm_budget must be positive");
    if (cfg->global_slots < 1 || cfg->global_slots > 256) return fail(RN_ERR_ARG, "global_slots must be in [1, 256]");
    rn_server *s = new (std::nothrow) rn_server();
    if (!s) return fail(RN_ERR_NOMEM, "allocating the server");
    s->guard = new (std::nothrow) BusyGuard(g);
    if (!s->guard || !s->guard->ok) {
        delete s->guard;
        delete s;
        return fail(RN_ERR_BUSY, "handle in use by another call");
    }
    s->g = g;
    s->cfg = *cfg;
    s->V = g->voff[cfg->graph + 1] - g->voff[cfg->graph];
    // first ball-size estimate: a planar road graph holds about 2 (theta / mean weight)^2
    // vertices within theta; refined from every theta-join that completes
    double wsum = 0;
    const int64_t a0 = g->aoff[cfg->graph], a1 = g->aoff[cfg->graph + 1];
    for (int64_t a = a0; a < a1; ++a) wsum += g->w[a];
    const double wmean = a1 > a0 ? std::max(1.0, wsum / static_cast<double>(a1 - a0)) : 1.0;
    s->c_ball = 2.0 / (wmean * wmean);
    rn_status st = RN_OK;
    hipError_t e = hipSetDevice(g->device);
    if (e != hipSuccess) st = hip_fail(e, "selecting the device");
    s->lanes.resize(static_cast<size_t>(cfg->lanes));
    for (Lane &L : s->lanes) {
        if (st != RN_OK) break;
        if ((e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&L.ev_state, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&L.ev_copy, hipEventDisableTiming)) != hipSuccess)
            st = hip_fail(e, "creating lane streams");
        L.ws.gslot_cap = static_cast<uint32_t>(cfg->global_slots);
        // a lane's global-tier slots are allocated here, when the server
        // starts, and not when a search first needs them: an allocation on
        // the request path would stall every lane (the bytes count in
        // rn_server_stats.device_bytes, outside the HBM budget)
        if (st == RN_OK) st = ensure_gslots(L.ws, g->Vmax, static_cast<uint32_t>(cfg->global_slots), L.stream);
    }
    if (st == RN_OK) {
        try {
            s->thr = std::thread(server_loop, s);
        } catch (...) {
            st = fail(RN_ERR_NOMEM, "starting the server thread");
        }
    }
    if (st != RN_OK) {
        const std::string msg = last_error();
        for (Lane &L : s->lanes) L.release();
        delete s->guard;
        delete s;
        return fail(st, msg);
    }
    *out = s;
    return RN_OK;
}

rn_status rn_server_submit(rn_server *s, const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, uint32_t theta,
                           int32_t k, int64_t *id) {
    if (!id) return fail(RN_ERR_ARG, "id is NULL");
    *id = 0;
    if (!s) return fail(RN_ERR_ARG, "server is NULL");
    if (nR < 1 || nS < 1 || !R || !S) return fail(RN_ERR_ARG, "R and S must each hold at least one vertex");
    if (static_cast<int64_t>(nR) + nS > s->V) return fail(RN_ERR_ARG, "R and S together exceed the vertex count");
    if (k < 0 || k > (1 << 24)) return fail(RN_ERR_ARG, "k must be 0 (theta-join) or in [1, 2^24]");
    if (theta > kMaxDist) return fail(RN_ERR_ARG, "theta must be <= 2^32 - 2");
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(RN_ERR_NOMEM, "allocating the request");
    try {
        r->R.assign(R, R + nR);
        r->S.assign(S, S + nS);
    } catch (...) {
        delete r;
        return fail(RN_ERR_NOMEM, "copying the request");
    }
    r->theta = theta;
    r->k = k;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return fail(RN_ERR_ARG, "the server is shutting down");
        }
        r->footprint = footprint(s, *r);
        r->heavy = work_estimate(s, *r) > kHeavyWork;
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->pending.push_back(r);
        s->stats.submitted += 1;
    }
    s->cv_work.notify_one();
    *id = r->id;
    return RN_OK;
}

rn_status rn_server_wait(rn_server *s, int64_t id, rn_pair *out, int64_t cap, int64_t *n_out, double *latency_ms) {
    if (n_out) *n_out = 0;
    if (!s) return fail(RN_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(RN_ERR_ARG, "unknown request id");
    Request *r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    const int64_t n = static_cast<int64_t>(r->result.size());
    if (n_out) *n_out = n;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    if (r->status != RN_OK) {
        const rn_status st = r->status;
        const std::string msg = r->err;
        s->reqs.erase(it);
        delete r;
        return fail(st, msg);
    }
    if (n > cap || (n > 0 && !out)) return fail(RN_ERR_CAPACITY, "output buffer too small");
    if (n) std::memcpy(out, r->result.data(), static_cast<size_t>(n) * sizeof(rn_pair));
    s->reqs.erase(it);
    delete r;
    return RN_OK;
}

rn_status rn_server_get_stats(rn_server *s, rn_server_stats *out) {
    if (!s || !out) return fail(RN_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return RN_OK;
}

void rn_server_free(rn_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->thr.joinable()) s->thr.join();
    (void)hipSetDevice(s->g->device);
    for (Lane &L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        L.release();
    }
    for (auto &kv : s->reqs) delete kv.second;
    delete s->guard;
    delete s;
}

}  // extern "C"
