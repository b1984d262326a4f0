// rn_partition.cpp -- the paper's heuristic graph partitioning (Section 3).
//
// One bisection (Algorithm 1) grows a left and a right cluster from two seed
// vertices.  Each cluster keeps a min-heap of the edges on its horizon, keyed
// by edge weight (not path length: this is a Prim-like growth).  Every step
// expands the cluster whose heap top is lighter after the smoothing of
// Equations (1)-(2):
//     w1' = |V1| / (|V1| + alpha |V2|) * w1,   w2' = |V2| / (alpha |V1| + |V2|) * w2,
// where |V1|, |V2| are the current cluster populations; alpha = 0 compares the
// raw weights, alpha = 1 scales each by its cluster's share of the population.
// The popped edge's far end joins the cluster if no cluster holds it yet, and
// its edges to unclaimed vertices enter that cluster's heap.  Edges that leave
// the part being split (the parent's cross-edges) are never followed.  Applied
// recursively this yields the partition hierarchy whose parts are far apart
// (Abstract; Section 1).
//
// Readings where the algorithm as printed is silent or inconsistent:
//  * a popped vertex joins a cluster only if it is in no cluster yet (the
//    printed test names only the expanding cluster, which would let a vertex
//    be claimed twice); the right-cluster branch records cross-edges towards
//    the left cluster (the printed test repeats "right"), and its heap pop sits
//    inside its own branch;
//  * ties: at equal smoothed weights the right cluster expands (the printed
//    test is a strict "better"); within a heap, ties go to the lower edge index;
//  * seeds: a double-sweep pseudo-diameter of the part (weighted shortest
//    paths from the part's lowest id to the farthest vertex a, then from a to
//    the farthest b; ties to the lowest id);
//  * stop rule: parts of at most max_leaf vertices are leaves;
//  * vertices reachable from neither seed inside the part (a disconnected
//    part) form a third child, split further like the others.
// Cross-edges are not stored: only the vertex order is used by the joins.
#include "rn_partition.h"

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <new>
#include <queue>
#include <thread>
#include <utility>

namespace rn {

namespace {

struct UGraph {  // undirected view: every arc x->y also listed as y->x
    std::vector<int64_t> off;
    std::vector<int32_t> adj;
    std::vector<uint32_t> wt;
};

void build_undirected(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                      UGraph &u) {
    const int64_t A = row_ptr[V];
    u.off.assign(static_cast<size_t>(V) + 1, 0);
    for (int32_t x = 0; x < V; ++x)
        for (int32_t a = row_ptr[x]; a < row_ptr[x + 1]; ++a) {
            u.off[x + 1]++;
            u.off[col[a] + 1]++;
        }
    for (int32_t x = 0; x < V; ++x) u.off[x + 1] += u.off[x];
    u.adj.resize(static_cast<size_t>(2 * A));
    u.wt.resize(static_cast<size_t>(2 * A));
    std::vector<int64_t> pos(u.off.begin(), u.off.end() - 1);
    for (int32_t x = 0; x < V; ++x)
        for (int32_t a = row_ptr[x]; a < row_ptr[x + 1]; ++a) {
            const int32_t y = col[a];
            u.adj[pos[x]] = y;
            u.wt[pos[x]++] = w[a];
            u.adj[pos[y]] = x;
            u.wt[pos[y]++] = w[a];
        }
}

struct Item {  // heap entry: edge weight, edge index, far end
    uint64_t w;
    int64_t idx;
    int32_t y;
};
struct ItemGreater {
    bool operator()(const Item &a, const Item &b) const {
        return a.w != b.w ? a.w > b.w : a.idx > b.idx;
    }
};
using MinHeap = std::priority_queue<Item, std::vector<Item>, ItemGreater>;

class Partitioner {
  public:
    Partitioner(int32_t V, const UGraph &g) : V_(V), g_(g) {
        stamp_.assign(static_cast<size_t>(V), 0);
        cl_.assign(static_cast<size_t>(V), 0);
        dist_.assign(static_cast<size_t>(V), UINT64_MAX);
    }

    // Farthest vertex (weighted, inside the stamped part) from s; ties to lowest id.
    // Parts being split at once are disjoint, so the per-vertex arrays are
    // shared by the worker threads; `touched` is the caller's own.
    int32_t farthest(int32_t s, uint32_t st, std::vector<int32_t> &touched_) {
        using P = std::pair<uint64_t, int32_t>;
        std::priority_queue<P, std::vector<P>, std::greater<P>> pq;
        touched_.clear();
        dist_[s] = 0;
        touched_.push_back(s);
        pq.push({0, s});
        uint64_t best_d = 0;
        int32_t best = s;
        while (!pq.empty()) {
            auto [d, x] = pq.top();
            pq.pop();
            if (d != dist_[x]) continue;
            if (d > best_d || (d == best_d && x < best)) {
                best_d = d;
                best = x;
            }
            for (int64_t e = g_.off[x]; e < g_.off[x + 1]; ++e) {
                const int32_t y = g_.adj[e];
                if (stamp_[y] != st) continue;
                const uint64_t nd = d + g_.wt[e];
                if (nd < dist_[y]) {
                    if (dist_[y] == UINT64_MAX) touched_.push_back(y);
                    dist_[y] = nd;
                    pq.push({nd, y});
                }
            }
        }
        for (int32_t x : touched_) dist_[x] = UINT64_MAX;
        return best;
    }

    // Stamp the part perm[b, e) with st and, if it is not connected (arcs
    // read as undirected edges), reorder it as its connected pieces, ordered
    // by their lowest vertex id, and return their ranges (true).  A connected
    // part returns false, stamped, for bisect.
    bool split_components(std::vector<int32_t> &perm, size_t b, size_t e, uint32_t st, std::vector<int32_t> &tmp,
                          std::vector<std::pair<size_t, size_t>> &ranges) {
        for (size_t i = b; i < e; ++i) {
            stamp_[perm[i]] = st;
            cl_[perm[i]] = 0;
        }
        // breadth-first pieces from the lowest unvisited id; cl_ marks visited vertices
        std::sort(perm.begin() + static_cast<std::ptrdiff_t>(b), perm.begin() + static_cast<std::ptrdiff_t>(e));
        tmp.clear();
        std::vector<size_t> starts;
        for (size_t i = b; i < e; ++i) {
            const int32_t s0 = perm[i];
            if (cl_[s0] != 0) continue;
            starts.push_back(tmp.size());
            cl_[s0] = 1;
            size_t head = tmp.size();
            tmp.push_back(s0);
            while (head < tmp.size()) {
                const int32_t x = tmp[head++];
                for (int64_t a = g_.off[x]; a < g_.off[x + 1]; ++a) {
                    const int32_t y = g_.adj[a];
                    if (stamp_[y] == st && cl_[y] == 0) {
                        cl_[y] = 1;
                        tmp.push_back(y);
                    }
                }
            }
            if (starts.size() == 1 && tmp.size() == e - b) break;   // connected
        }
        for (size_t i = b; i < e; ++i) cl_[perm[i]] = 0;
        if (starts.size() <= 1) return false;
        std::copy(tmp.begin(), tmp.end(), perm.begin() + static_cast<std::ptrdiff_t>(b));
        for (size_t c = 0; c < starts.size(); ++c)
            ranges.emplace_back(b + starts[c], b + (c + 1 < starts.size() ? starts[c + 1] : tmp.size()));
        return true;
    }

    void push_edges(MinHeap &h, int32_t x, uint32_t st) {
        for (int64_t e = g_.off[x]; e < g_.off[x + 1]; ++e) {
            const int32_t y = g_.adj[e];
            if (stamp_[y] == st && cl_[y] == 0) h.push({g_.wt[e], e, y});
        }
    }

    // Algorithm 1 on the part perm[b, e): sets cl_ to 1 (left), 2 (right) or 0.
    // A cluster holding `cap` vertices stops growing (the other one, or a third
    // child of what neither reaches, takes the rest).
    void bisect(const std::vector<int32_t> &perm, size_t b, size_t e, uint32_t st, float alpha, size_t cap,
                std::vector<int32_t> &touched) {
        int32_t lowest = perm[b];
        for (size_t i = b; i < e; ++i) lowest = std::min(lowest, perm[i]);
        const int32_t sa = farthest(lowest, st, touched);
        int32_t sb = farthest(sa, st, touched);
        if (sb == sa) {  // seed component is a single vertex: take any other vertex
            sb = perm[b] != sa ? perm[b] : perm[b + 1];
        }
        for (size_t i = b; i < e; ++i) cl_[perm[i]] = 0;
        MinHeap L, R;
        cl_[sa] = 1;
        cl_[sb] = 2;
        double n1 = 1.0, n2 = 1.0;
        push_edges(L, sa, st);
        push_edges(R, sb, st);
        const double al = alpha;
        const double capd = static_cast<double>(cap);
        while (true) {
            const bool lok = !L.empty() && n1 < capd, rok = !R.empty() && n2 < capd;
            if (!lok && !rok) break;
            bool left;
            if (!rok) {
                left = true;
            } else if (!lok) {
                left = false;
            } else {
                const double w1 = n1 / (n1 + al * n2) * static_cast<double>(L.top().w);
                const double w2 = n2 / (al * n1 + n2) * static_cast<double>(R.top().w);
                left = w1 < w2;
            }
            MinHeap &h = left ? L : R;
            const Item it = h.top();
            h.pop();
            if (cl_[it.y] != 0) continue;
            cl_[it.y] = left ? 1 : 2;
            (left ? n1 : n2) += 1.0;
            push_edges(h, it.y, st);
        }
    }

    // The recursion: parts are split by several host threads at once (a
    // part's split depends only on its own vertices, so the result does not
    // depend on the schedule); leaves are numbered afterwards by a
    // left-to-right walk of the tree.
    void run(float alpha, int32_t max_leaf, std::vector<int32_t> &part, std::vector<int32_t> &order) {
        struct Node {
            size_t b, e;
            int32_t first;      // first child (children are consecutive), -1 for a leaf
            int32_t nchild;
        };
        std::vector<int32_t> perm(static_cast<size_t>(V_));
        for (int32_t i = 0; i < V_; ++i) perm[i] = i;
        std::vector<Node> nodes;
        // every split makes at least two non-empty children, so a tree over V
        // vertices has fewer than 2V nodes: reserved once, never reallocated
        // while workers read it
        nodes.reserve(static_cast<size_t>(V_) * 2 + 2);
        nodes.push_back(Node{0, perm.size(), -1, 0});
        std::mutex mu;
        std::condition_variable cv;
        std::vector<int32_t> todo{0};
        size_t busy = 0;
        std::atomic<uint32_t> next_stamp{1};
        bool failed = false;
        auto worker = [&]() {
            std::vector<int32_t> tmp, touched;
            try {
                while (true) {
                    int32_t id;
                    size_t b, e;
                    {
                        std::unique_lock<std::mutex> lk(mu);
                        cv.wait(lk, [&] { return !todo.empty() || busy == 0 || failed; });
                        if (todo.empty() || failed) return;
                        id = todo.back();
                        todo.pop_back();
                        ++busy;
                        b = nodes[static_cast<size_t>(id)].b;
                        e = nodes[static_cast<size_t>(id)].e;
                    }
                    std::vector<std::pair<size_t, size_t>> ranges;
                    if (e - b <= static_cast<size_t>(max_leaf) || e - b < 2) {
                        std::sort(perm.begin() + static_cast<std::ptrdiff_t>(b),
                                  perm.begin() + static_cast<std::ptrdiff_t>(e));
                    } else if (const uint32_t st = next_stamp++; split_components(perm, b, e, st, tmp, ranges)) {
                        // a disconnected part: its connected pieces are its children
                    } else {
                        // parts of more than two leaves: neither cluster takes more
                        // than 3/4 of the part, which bounds the depth of the
                        // recursion (with alpha = 0 nothing evens the clusters out,
                        // and lopsided splits peel a few vertices off a large part
                        // level after level)
                        const size_t n = e - b;
                        const size_t ml = static_cast<size_t>(max_leaf);
                        const size_t cap = n > ml + ml / 4 + 1 ? (3 * n + 3) / 4 : n;
                        bisect(perm, b, e, st, alpha, cap, touched);
                        tmp.clear();
                        for (int c : {1, 2, 0})
                            for (size_t i = b; i < e; ++i)
                                if (cl_[perm[i]] == c) tmp.push_back(perm[i]);
                        size_t n1 = 0, n2 = 0;
                        for (size_t i = b; i < e; ++i) {
                            n1 += cl_[perm[i]] == 1;
                            n2 += cl_[perm[i]] == 2;
                        }
                        std::copy(tmp.begin(), tmp.end(), perm.begin() + static_cast<std::ptrdiff_t>(b));
                        const size_t m1 = b + n1, m2 = m1 + n2;
                        const size_t cut[4] = {b, m1, m2, e};
                        for (int c = 0; c < 3; ++c)
                            if (cut[c + 1] > cut[c]) ranges.emplace_back(cut[c], cut[c + 1]);
                    }
                    std::lock_guard<std::mutex> lk(mu);
                    Node &nd = nodes[static_cast<size_t>(id)];
                    nd.first = ranges.empty() ? -1 : static_cast<int32_t>(nodes.size());
                    nd.nchild = static_cast<int32_t>(ranges.size());
                    for (const auto &r : ranges) {
                        todo.push_back(static_cast<int32_t>(nodes.size()));
                        nodes.push_back(Node{r.first, r.second, -1, 0});
                    }
                    --busy;
                    cv.notify_all();
                }
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                failed = true;
                cv.notify_all();
            }
        };
        const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; ++t) pool.emplace_back(worker);
        worker();
        for (auto &t : pool) t.join();
        if (failed) throw std::bad_alloc();
        // leaves in a left-to-right walk of the tree
        order.clear();
        order.reserve(static_cast<size_t>(V_));
        part.assign(static_cast<size_t>(V_), 0);
        int32_t leaf = 0;
        std::vector<int32_t> stack{0};
        while (!stack.empty()) {
            const Node &nd = nodes[static_cast<size_t>(stack.back())];
            stack.pop_back();
            if (nd.first < 0) {
                for (size_t i = nd.b; i < nd.e; ++i) {
                    part[perm[i]] = leaf;
                    order.push_back(perm[i]);
                }
                ++leaf;
                continue;
            }
            for (int32_t c = nd.nchild - 1; c >= 0; --c) stack.push_back(nd.first + c);
        }
    }

  private:
    int32_t V_;
    const UGraph &g_;
    std::vector<uint32_t> stamp_;
    std::vector<uint8_t> cl_;
    std::vector<uint64_t> dist_;
};

}  // namespace

bool partition_graph(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                     float alpha, int32_t max_leaf, std::vector<int32_t> &part,
                     std::vector<int32_t> &order, std::string &msg) {
    try {
        UGraph u;
        build_undirected(V, row_ptr, col, w, u);
        Partitioner p(V, u);
        p.run(alpha, max_leaf, part, order);
    } catch (const std::bad_alloc &) {
        msg = "out of host memory while partitioning";
        return false;
    }
    return true;
}

}  // namespace rn
