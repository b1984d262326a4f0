"""Pins of the CPU oracle against things other than itself.

Each check rests on a fact fixed independently of the oracle's code:
  * brute force: Floyd-Warshall distances on tiny graphs (numpy min-plus), and
    the definitions of both joins evaluated on them (Abstract; Section 1);
  * a library routine: scipy.sparse.csgraph.dijkstra with a distance limit;
  * a closed form: on a full lattice with uniform weight c,
    dist = c * (|di| + |dj|);
  * invariants: symmetry on undirected graphs, the triangle inequality,
    monotonicity in theta and k, the k-closest pairs being the theta-join
    taken at theta = d_k (Section 4: an unbounded k gives the theta-join), and
    the one-hop special case d_k < 2 w_min;
  * the shortest-path optimality (Bellman) certificate;
  * a hand-derived example (tests/golden/hand_graph.json).
Planted mistakes in copies of the oracle source (test_mutants_are_caught)
show that these pins catch dropped terms, wrong bounds, wrong orders and
transposed outputs.
"""
import json
import os
import shutil

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_graph.json")
INF = np.iinfo(np.uint64).max


# ----------------------------------------------------------------- brute force
def floyd_warshall(g):
    """All-pairs distances (uint64, INF unreachable) by the Floyd-Warshall recurrence."""
    V = g.V
    D = np.full((V, V), INF, dtype=np.uint64)
    np.fill_diagonal(D, 0)
    src = np.repeat(np.arange(V), np.diff(g.row_ptr))
    for s, t, w in zip(src, g.col, g.w.astype(np.uint64)):
        if w < D[s, t]:
            D[s, t] = w
    for k in range(V):
        via = np.where((D[:, k:k + 1] == INF) | (D[k:k + 1, :] == INF), INF,
                       D[:, k:k + 1] + D[k:k + 1, :])
        D = np.minimum(D, via)
    return D


def brute_pairs(D, R, S, theta=None):
    """Every reachable (u, v, d) with u in R, v in S (d <= theta if given), sorted by (d, u, v)."""
    rows = []
    for u in R:
        for v in S:
            d = D[u, v]
            if d < 0xFFFFFFFF and (theta is None or d <= theta):
                rows.append((int(d), int(u), int(v)))
    rows.sort()
    return [(u, v, d) for d, u, v in rows]


def as_list(pairs):
    return [(int(p["u"]), int(p["v"]), int(p["dist"])) for p in pairs]


def tiny_graphs(rg):
    out = []
    for seed in range(4):
        out.append(rg.random_digraph(14, 40, seed, wmin=1, wmax=20, zero_frac=0.15))
    out.append(rg.random_digraph(20, 25, 9, wmin=0, wmax=5))          # sparse: unreachable pairs
    for seed in range(3):
        out.append(rg.road_graph(6, seed, p_drop=0.5, keep_lcc=False))  # several components
    out.append(rg.road_graph(9, 3))
    return out


def split_sets(V, seed, nR, nS):
    rng = np.random.default_rng(seed)
    idx = rng.permutation(V)
    return idx[:nR].astype(np.int32), idx[nR:nR + nS].astype(np.int32)


# ----------------------------------------------------------------- pin groups
def check_brute_force(orc, rg, lib=None):
    for gi, g in enumerate(tiny_graphs(rg)):
        D = floyd_warshall(g)
        for s in range(g.V):
            d = orc.sssp(g, s, lib=lib).astype(np.uint64)
            want = np.where(D[s] >= 0xFFFFFFFF, 0xFFFFFFFF, D[s])
            assert np.array_equal(d, want), f"graph {gi} source {s}"
        R, S = split_sets(g.V, gi, g.V // 3, g.V // 3)
        finite = D[np.ix_(R, S)][D[np.ix_(R, S)] < 0xFFFFFFFF]
        thetas = [0, 1] + sorted(set(int(x) for x in finite))[:6] + [10 ** 6]
        for theta in thetas:
            r = orc.dist_join(g, R, S, theta, threads=2, lib=lib)
            assert as_list(r.pairs) == brute_pairs(D, R, S, theta), f"graph {gi} theta {theta}"
            reach = D[np.ix_(R, np.arange(g.V))] <= theta
            assert r.settled == int(reach.sum())
            assert r.arcs == int((reach * np.diff(g.row_ptr)[None, :]).sum())
        allp = brute_pairs(D, R, S)
        for k in (1, 2, 3, 5, len(allp), len(allp) + 3):
            if k < 1:
                continue
            assert as_list(orc.kcp_join(g, R, S, k, lib=lib)) == allp[:k], f"graph {gi} k {k}"


def check_golden(orc, rg, lib=None):
    d = json.load(open(GOLDEN))
    a = np.array(d["arcs"])
    g = rg.from_edges(d["V"], a[:, 0], a[:, 1], a[:, 2], symmetric=False)
    for c in d["cases"]:
        if c["kind"] == "join":
            got = as_list(orc.dist_join(g, c["R"], c["S"], c["theta"], lib=lib).pairs)
        else:
            got = as_list(orc.kcp_join(g, c["R"], c["S"], c["k"], lib=lib))
        assert got == [tuple(p) for p in c["pairs"]], c


def check_lattice(orc, rg, lib=None, side=48, c=7):
    g = rg.full_lattice(side, c)
    R, S = rg.sample_disjoint(g.V, 200, 300, 11)
    ri, rj = np.divmod(R.astype(np.int64), side)
    si, sj = np.divmod(S.astype(np.int64), side)
    dist = c * (np.abs(ri[:, None] - si[None, :]) + np.abs(rj[:, None] - sj[None, :]))
    for theta in (0, c * 3, c * 10, c * 10 + 3):
        want = sorted((int(dist[a, b]), int(R[a]), int(S[b]))
                      for a, b in zip(*np.nonzero(dist <= theta)))
        got = as_list(orc.dist_join(g, R, S, theta, threads=3, lib=lib).pairs)
        assert got == [(u, v, d) for d, u, v in want], theta
    allp = sorted((int(dist[a, b]), int(R[a]), int(S[b])) for a in range(len(R)) for b in range(len(S)))
    for k in (1, 7, 64, 500):
        assert as_list(orc.kcp_join(g, R, S, k, lib=lib)) == [(u, v, d) for d, u, v in allp[:k]], k


def check_scipy(orc, rg, lib=None):
    g = rg.road_graph(64, 0)
    R, S = rg.sample_disjoint(g.V, 64, 64, 1)
    m = sp.csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.V, g.V))
    for theta in (700, 1500, 2600):
        D = dijkstra(m, directed=True, indices=R, limit=theta)
        sub = D[:, S]
        want = sorted((int(sub[a, b]), int(R[a]), int(S[b])) for a, b in zip(*np.nonzero(sub <= theta)))
        r = orc.dist_join(g, R, S, theta, lib=lib)
        assert as_list(r.pairs) == [(u, v, d) for d, u, v in want], theta
        assert r.settled == int((D <= theta).sum())
        assert r.arcs == int(((D <= theta) * np.diff(g.row_ptr)[None, :]).sum())


ALL_CHECKS = [check_brute_force, check_golden, check_lattice, check_scipy]


# ----------------------------------------------------------------- tests
def test_brute_force_tiny_graphs(orc, rg):
    check_brute_force(orc, rg)


def test_golden_hand_example(orc, rg):
    check_golden(orc, rg)


def test_lattice_closed_form(orc, rg):
    check_lattice(orc, rg)


def test_scipy_dijkstra(orc, rg):
    check_scipy(orc, rg)


def test_symmetry_on_undirected_graph(orc, rg):
    g = rg.road_graph(64, 0)
    R, S = rg.sample_disjoint(g.V, 80, 90, 4)
    a = as_list(orc.dist_join(g, R, S, 1800).pairs)
    b = as_list(orc.dist_join(g, S, R, 1800).pairs)
    assert sorted(a) == sorted((v, u, d) for u, v, d in b)


def test_triangle_inequality(orc, rg):
    g = rg.road_graph(64, 0)
    rng = np.random.default_rng(5)
    pts = rng.choice(g.V, size=24, replace=False)
    D = np.stack([orc.sssp(g, int(s)).astype(np.int64) for s in pts])[:, pts]
    for i in range(len(pts)):
        for j in range(len(pts)):
            assert D[i, j] <= (D[i, :] + D[:, j]).min()
    assert np.array_equal(D, D.T)


def test_bellman_certificate(orc, rg):
    g = rg.road_graph(64, 0)
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    w = g.w.astype(np.int64)
    for s in (0, 1234, 4000):
        for cutoff in (900, 0xFFFFFFFE):
            d = orc.sssp(g, s, cutoff).astype(np.int64)
            reached = d != 0xFFFFFFFF
            assert d[s] == 0
            # relaxed: no arc can improve a reached target within the cutoff
            cand = d[src] + w
            ok = ~reached[src] | (cand > cutoff) | (reached[g.col] & (d[g.col] <= cand))
            assert ok.all()
            # tight: every reached vertex but s has an in-arc achieving its distance
            best = np.full(g.V, np.iinfo(np.int64).max)
            m = reached[src]
            np.minimum.at(best, g.col[m], cand[m])
            r = reached.copy()
            r[s] = False
            assert np.array_equal(best[r], d[r])


def test_monotone_in_theta_and_k(orc, rg):
    g = rg.road_graph(64, 0)
    R, S = rg.sample_disjoint(g.V, 64, 64, 1)
    prev = set()
    for theta in (300, 800, 1500, 2200):
        cur = set(as_list(orc.dist_join(g, R, S, theta).pairs))
        assert prev <= cur
        prev = cur
    big = as_list(orc.kcp_join(g, R, S, 300))
    for k in (1, 16, 100, 299):
        assert as_list(orc.kcp_join(g, R, S, k)) == big[:k]


def test_kcp_equals_join_prefix_at_dk(orc, rg):
    g = rg.road_graph(64, 0)
    for seed, k in ((1, 16), (2, 100), (3, 1000)):
        R, S = rg.sample_disjoint(g.V, 64, 64, seed)
        kc = as_list(orc.kcp_join(g, R, S, k))
        assert len(kc) == k
        dk = kc[-1][2]
        join = as_list(orc.dist_join(g, R, S, dk).pairs)
        assert join[:k] == kc
        assert all(d == dk for _, _, d in join[k:])


def test_kcp_one_hop_special_case(orc, rg):
    g = rg.road_graph(128, 0)
    R, S = rg.sample_clustered(g, 2048, 2048, 3)
    inS = np.zeros(g.V, bool)
    inS[S] = True
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    isR = np.zeros(g.V, bool)
    isR[R] = True
    m = isR[src] & inS[g.col]
    direct = sorted(zip(g.w[m].astype(int), src[m].astype(int), g.col[m].astype(int)))
    wmin = int(g.w.min())
    for k in (1, 10, 40):
        kc = as_list(orc.kcp_join(g, R, S, k))
        assert kc[-1][2] < 2 * wmin, "instance does not satisfy d_k < 2 w_min"
        assert kc == [(u, v, d) for d, u, v in direct[:k]]


def test_rejects_bad_ids(orc, rg):
    g = rg.road_graph(8, 0)
    with pytest.raises(ValueError):
        orc.dist_join(g, [0, g.V], [1], 10)
    with pytest.raises(ValueError):
        orc.kcp_join(g, [0], [1], 0)


# ----------------------------------------------------------------- planted mistakes
MUTANTS = {
    "theta_exclusive": ("if (it.d > theta) break;", "if (it.d >= theta) break;"),
    "weight_halved": ("uint64_t nd = it.d + s->w[a];", "uint64_t nd = it.d + s->w[a] / 2;"),
    "last_arc_dropped": ("for (int32_t a = s->row_ptr[x]; a < s->row_ptr[x + 1]; a++) {",
                         "for (int32_t a = s->row_ptr[x]; a < s->row_ptr[x + 1] - 1; a++) {"),
    "order_v_before_u": ("    if (a->u != b->u) return a->u < b->u;\n    return a->v < b->v;",
                         "    if (a->v != b->v) return a->v < b->v;\n    return a->u < b->u;"),
    "kcp_drops_ties": ("if (nd > ph_bound(&h) || nd >= ws.dist[y]) continue;",
                       "if (nd >= ph_bound(&h) || nd >= ws.dist[y]) continue;"),
    "arc_count_wrong": ("*arcs += s->row_ptr[x + 1] - s->row_ptr[x];", "*arcs += 1;"),
    "pair_transposed": ("if (inS[x] && pv_push(out, u, x, (uint32_t)it.d)) return -1;",
                        "if (inS[x] && pv_push(out, x, u, (uint32_t)it.d)) return -1;"),
    "heap_order_flipped": ("        if (h->a[p].d <= d) break;", "        if (h->a[p].d >= d) break;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_are_caught(orc, rg, tmp_path, name):
    old, new = MUTANTS[name]
    src = open(orc.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    msrc = tmp_path / "rn_oracle_mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = orc.open_library(orc.build(str(msrc), str(tmp_path / f"liborc_{name}.so")))
    caught = []
    for check in ALL_CHECKS:
        try:
            check(orc, rg, lib=lib)
        except AssertionError:
            caught.append(check.__name__)
    assert caught, f"mutant {name} passed every pin"
