"""Pins of the oracle's join of objects on edges (Section 1: objects moving
along the network's edges, given by their distances from the two ends of
their edge, taking the place of R or S nodes).

The oracle evaluates the reading by its end-to-end formula (leave the
object's edge at an end, follow the network, enter the other object's edge
at an end, or stay on a shared edge).  The pins here compute the same
distances another way: every object is inserted into its edge as a vertex
(the edge's arcs split at the objects' positions), and distances between
the new vertices come from Floyd-Warshall on tiny graphs or from scipy's
Dijkstra on a road graph; plus a small example worked by hand.  Planted
mistakes in copies of the oracle's object code must fail one of them.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

from test_oracle_pins import floyd_warshall

UNREACH = 0xFFFFFFFF


def tail_of(g, e):
    return int(np.searchsorted(g.row_ptr, e, side="right") - 1)


def place(g, e, o):
    """The edge an object (arc e, distance o from e's tail) is on: (f, s,
    twin of f or -1), f the arc naming the edge and s the distance from f's tail."""
    a, b, w = tail_of(g, e), int(g.col[e]), int(g.w[e])
    row_a = range(int(g.row_ptr[a]), int(g.row_ptr[a + 1]))
    row_b = range(int(g.row_ptr[b]), int(g.row_ptr[b + 1]))
    ec = next(x for x in row_a if g.col[x] == b and g.w[x] == w)
    tw = next((x for x in row_b if g.col[x] == a and g.w[x] == w and x != ec), -1)
    if tw >= 0 and tw < ec:
        return tw, w - o, ec
    return ec, o, tw


def subdivide(g, objects):
    """The graph with object i inserted as vertex V + i: each object's edge
    (its arc f and, on a two-way road, f's twin) is split at the objects'
    positions.  Returns (V', src, dst, w)."""
    V = g.V
    on = {}                      # f -> [(s, vertex)]
    twin = {}
    for i, (e, o) in enumerate(objects):
        f, s, tw = place(g, int(e), int(o))
        on.setdefault(f, []).append((s, V + i))
        twin[f] = tw
    replaced = set(on) | {t for f, t in twin.items() if t >= 0}
    src, dst, ww = [], [], []
    tails = np.repeat(np.arange(V), np.diff(g.row_ptr))
    for x in range(g.A):
        if x not in replaced:
            src.append(int(tails[x])); dst.append(int(g.col[x])); ww.append(int(g.w[x]))
    for f, lst in on.items():
        lst.sort()
        a, b, w = int(tails[f]), int(g.col[f]), int(g.w[f])
        chain = [(0, a)] + lst + [(w, b)]
        for (s0, u), (s1, v) in zip(chain, chain[1:]):
            src.append(u); dst.append(v); ww.append(s1 - s0)
            if twin[f] >= 0:
                src.append(v); dst.append(u); ww.append(s1 - s0)
    return V + len(objects), np.array(src), np.array(dst), np.array(ww, dtype=np.int64)


def as_graph(rg, Vn, src, dst, w):
    return rg.from_edges(Vn, src, dst, w.astype(np.uint32), symmetric=False)


def as_list(pairs):
    return [(int(p["u"]), int(p["v"]), int(p["dist"])) for p in pairs]


def want_pairs(D, nR, nS, theta):
    rows = sorted((int(D[i, nR + j]), i, j) for i in range(nR) for j in range(nS)
                  if D[i, nR + j] < UNREACH and D[i, nR + j] <= theta)
    return [(i, j, d) for d, i, j in rows]


def random_objects(g, n, rng, share=None):
    """n objects: random arcs and offsets, including both ends of an edge,
    and (share) some on the arcs of another object list."""
    arcs = rng.integers(0, g.A, size=n)
    if share is not None and len(share):
        pick = rng.random(n) < 0.3
        arcs[pick] = rng.choice(share, size=int(pick.sum()))
    w = g.w[arcs].astype(np.int64)
    off = (rng.random(n) * (w + 1)).astype(np.int64)
    off = np.minimum(off, w)
    off[rng.random(n) < 0.1] = 0
    ends = rng.random(n) < 0.1
    off[ends] = w[ends]
    return arcs.astype(np.int32), off.astype(np.uint32)


def tiny_cases(rg):
    gs = [rg.random_digraph(12, 36, s, wmin=0, wmax=20, zero_frac=0.1) for s in range(3)]
    gs += [rg.road_graph(5, s, p_drop=0.3, keep_lcc=False) for s in range(2)]
    gs.append(rg.road_graph(7, 4))
    return gs


# ----------------------------------------------------------------- pin groups
def check_objects_brute(orc, rg, lib=None):
    for gi, g in enumerate(tiny_cases(rg)):
        rng = np.random.default_rng(50 + gi)
        Ra, Ro = random_objects(g, 6, rng)
        Sa, So = random_objects(g, 7, rng, share=Ra)
        objs = list(zip(Ra, Ro)) + list(zip(Sa, So))
        Vn, s_, d_, w_ = subdivide(g, objs)
        D = floyd_warshall(as_graph(rg, Vn, s_, d_, w_))[g.V:, g.V:]
        finite = sorted(set(int(x) for x in D[:6, 6:].ravel() if x < UNREACH))
        for theta in [0, 1] + finite[:5] + [10 ** 6]:
            got = as_list(orc.object_join(g, Ra, Ro, Sa, So, theta, lib=lib))
            assert got == want_pairs(D, 6, 7, theta), (gi, theta)


def check_objects_scipy(orc, rg, lib=None):
    g = rg.road_graph(24, 2)
    rng = np.random.default_rng(7)
    Ra, Ro = random_objects(g, 40, rng)
    Sa, So = random_objects(g, 50, rng, share=Ra)
    objs = list(zip(Ra, Ro)) + list(zip(Sa, So))
    Vn, s_, d_, w_ = subdivide(g, objs)
    # scipy drops explicit zeros and sums duplicate entries: keep the lightest
    # of parallel arcs, and add eps = 1 / (8 V') to every weight, which keeps
    # zero-length arcs (objects at an edge end or at one spot) and lifts any
    # simple path by less than 1/8, so the floor of a float distance is the
    # integer one
    best = {}
    for a, b, c in zip(s_, d_, w_):
        best[(int(a), int(b))] = min(best.get((int(a), int(b)), int(c)), int(c))
    eps = 1.0 / (8 * Vn)
    keys = list(best)
    m = sp.csr_matrix(([best[k] + eps for k in keys], ([k[0] for k in keys], [k[1] for k in keys])),
                      shape=(Vn, Vn))
    D = np.floor(dijkstra(m, directed=True, indices=np.arange(g.V, g.V + 40))[:, g.V + 40:])
    for theta in (0, 150, 600, 1500, 4000):
        rows = sorted((int(D[i, j]), i, j) for i in range(40) for j in range(50) if D[i, j] <= theta)
        got = as_list(orc.object_join(g, Ra, Ro, Sa, So, theta, lib=lib))
        assert got == [(i, j, d) for d, i, j in rows], theta


def check_objects_hand(orc, rg, lib=None):
    # a two-way road 0 -(10)- 1 -(6)- 2 and a one-way arc 2 -> 3 of weight 5.
    # Arcs (from_edges sorts by tail, head): 0: 0->1, 1: 1->0, 2: 1->2, 3: 2->1, 4: 2->3.
    g = rg.from_edges(4, [0, 1, 1, 2, 2], [1, 0, 2, 1, 3], np.array([10, 10, 6, 6, 5], np.uint32),
                      symmetric=False)
    # R: p0 on 0->1 at 3 (7 from node 1); p1 on 2->3 at 1 (one-way: only 3 is reachable)
    # S: q0 on 1->0 at 2 (the same road as p0, 8 from node 0); q1 on 1->2 at 4;
    #    q2 on 2->3 at 4 (ahead of p1 on the one-way arc); q3 on 2->3 at 0 (behind p1)
    Ra, Ro = [0, 4], [3, 1]
    Sa, So = [1, 2, 4, 4], [2, 4, 4, 0]
    # by hand: p0-q0 along the road: 8 - 3 = 5; p0-q1: 7 to node 1, then 4 = 11;
    # p0-q2: 7 + 6 to node 2, then 4 = 17; p0-q3: 13 to node 2, 0 more = 13;
    # p1: leaves only forward, to node 3, which leads nowhere: q2 is 3 ahead on
    # the same arc, q3 is behind it (unreachable)
    want = sorted([(5, 0, 0), (11, 0, 1), (17, 0, 2), (13, 0, 3), (3, 1, 2)])
    got = as_list(orc.object_join(g, Ra, Ro, Sa, So, 100, lib=lib))
    assert got == [(i, j, d) for d, i, j in want]
    got = as_list(orc.object_join(g, Ra, Ro, Sa, So, 11, lib=lib))
    assert got == [(i, j, d) for d, i, j in want if d <= 11]


OBJECT_CHECKS = [check_objects_brute, check_objects_scipy, check_objects_hand]


def test_objects_brute_force(orc, rg):
    check_objects_brute(orc, rg)


def test_objects_scipy_on_subdivided_road(orc, rg):
    check_objects_scipy(orc, rg)


def test_objects_hand_example(orc, rg):
    check_objects_hand(orc, rg)


def test_objects_reject_bad_offsets(orc, rg):
    g = rg.road_graph(5, 0)
    with pytest.raises(ValueError):
        orc.object_join(g, [0], [int(g.w[0]) + 1], [1], [0], 100)
    with pytest.raises(ValueError):
        orc.object_join(g, [g.A], [0], [1], [0], 100)


OBJECT_MUTANTS = {
    "one_way_everywhere": ("    ob->two_way = tw >= 0;", "    ob->two_way = 0;"),
    "offset_from_head": ("        ob->f = ec; ob->s = o; ob->tail = a; ob->head = b;",
                         "        ob->f = ec; ob->s = wt - o; ob->tail = a; ob->head = b;"),
    "shared_edge_ignored": ("            if (q->f == p->f) {", "            if (q->f == p->f && 0) {"),
    "enter_from_head_only": (
        "            if (ws.dist[q->tail] != ORC_UNREACH && ws.dist[q->tail] + q->s < best) best = ws.dist[q->tail] + q->s;",
        "            if (0) best = ws.dist[q->tail] + q->s;"),
    "twin_not_merged": ("    if (tw >= 0 && tw < ec) {", "    if (0) {"),
}


@pytest.mark.parametrize("name", sorted(OBJECT_MUTANTS))
def test_object_mutants_are_caught(orc, rg, tmp_path, name):
    old, new = OBJECT_MUTANTS[name]
    src = open(orc.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    msrc = tmp_path / "rn_oracle_mutant.c"
    msrc.write_text(src.replace(old, new))
    lib = orc.open_library(orc.build(str(msrc), str(tmp_path / f"liborc_{name}.so")))
    caught = []
    for check in OBJECT_CHECKS:
        try:
            check(orc, rg, lib=lib)
        except (AssertionError, ValueError):
            caught.append(check.__name__)
    assert caught, f"mutant {name} passed every pin"
