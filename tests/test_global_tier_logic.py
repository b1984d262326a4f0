"""Host-side check of the global tier's round logic (the near-far search of
searches that outgrow every on-chip table): a Python emulation of one block's
rounds -- one 64-bit word per vertex, (distance, 1 + round of its last
improvement), far-list membership without a bitmap, bucket splits that mark
vertices dropped for lying beyond a falling bound -- with each chunk's
relaxations applied in random order, as the block's threads may apply them.
Distances within the bound must equal Dijkstra's (scipy), and the frontier and
far list must never hold a vertex twice.  A planted mistake (a vertex counted
as queued whenever it was improved this round, also when that improvement went
to the far list) must fail."""
import random

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

INF = 0xFFFFFFFF
CHUNK = 64


def emulate(g, s, gdelta, bound_of, rng, planted=False):
    word = {s: (0, 1)}
    W = lambda v: word.get(v, (INF, INF))
    cur, far, thr, rnd = [s], [], gdelta, 1
    while True:
        bound = bound_of(rnd)
        if not cur:
            if not far:
                break
            told = thr
            cand = [W(v)[0] for v in far if thr <= W(v)[0] <= bound]
            if cand:
                thr = (min(cand) // gdelta + 1) * gdelta
            kept = []
            for v in far:
                d = W(v)[0]
                if d != INF and d > bound:
                    word[v] = (d, 0)            # dropped beyond the bound: marked
                if told <= d < thr and d <= bound:
                    cur.append(v)
                if thr <= d <= bound:
                    kept.append(v)
            far = kept
            continue
        nxt = []
        for c0 in range(0, len(cur), CHUNK):
            chunk = cur[c0:c0 + CHUNK]
            rel = []
            for x in chunk:
                dx = W(x)[0]                     # read when the chunk starts
                for e in range(g.row_ptr[x], g.row_ptr[x + 1]):
                    rel.append((min(INF, dx + int(g.w[e])), int(g.col[e])))
            rng.shuffle(rel)
            for nd, y in rel:
                if not (nd <= bound and nd < INF):
                    continue
                od, otag = W(y)
                if (nd, rnd + 1) < (od, otag):
                    word[y] = (nd, rnd + 1)      # the 64-bit atomicMin
                imp = nd < od
                queued = otag == rnd + 1 and (planted or od < thr)
                if imp and nd < thr and not queued:
                    nxt.append(y)
                if imp and nd >= thr and (od == INF or otag == 0):
                    far.append(y)
        assert len(nxt) == len(set(nxt)), "a vertex queued twice in one round"
        assert len(far) == len(set(far)), "a vertex twice on the far list"
        cur, rnd = nxt, rnd + 1
    return {v: d for v, (d, _) in word.items()}


def scipy_dist(g, s):
    V = g.V
    best = {}
    for x in range(V):
        for e in range(g.row_ptr[x], g.row_ptr[x + 1]):
            k = (x, int(g.col[e]))
            best[k] = min(best.get(k, int(g.w[e])), int(g.w[e]))
    eps = 1.0 / (4 * V)
    keys = list(best)
    m = sp.csr_matrix(([best[k] + eps for k in keys], ([k[0] for k in keys], [k[1] for k in keys])), shape=(V, V))
    d = dijkstra(m, directed=True, indices=s)
    return [INF if not np.isfinite(x) else int(np.floor(x)) for x in d]


def cases(rg):
    out = []
    for t in range(12):
        if t % 3 == 0:
            g = rg.road_graph(20, t)
        elif t % 3 == 1:
            g = rg.random_digraph(250, 1000, t, wmin=0, wmax=60, zero_frac=0.1)
        else:
            g = rg.road_graph(14, t, p_drop=0.3, keep_lcc=False)
        out.append((t, g))
    return out


def run_cases(rg, planted):
    rng = random.Random(7)
    wrong = 0
    for t, g in cases(rg):
        s = rng.randrange(g.V)
        d = scipy_dist(g, s)
        fin = sorted(x for x in d if x < INF)
        B = fin[len(fin) * 2 // 3] if fin else 0
        gd = max(1, int((8 if t % 2 else 1) * np.mean(g.w)))
        if t % 4 < 2:
            bound_of = lambda r, B=B: B
        else:
            bound_of = lambda r, B=B: INF - 1 if r < 3 else max(B, (INF - 1) // (r * r))
        got = emulate(g, s, gd, bound_of, rng, planted)
        wrong += any(got.get(v, INF) != d[v] for v in range(g.V) if d[v] <= B)
    return wrong


def test_round_logic_matches_dijkstra(rg):
    assert run_cases(rg, planted=False) == 0


def test_planted_queue_mistake_is_caught(rg):
    assert run_cases(rg, planted=True) > 0
