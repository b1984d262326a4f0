"""Host partitioner (Section 3, Algorithm 1 with Equations (1)-(2)).

Pins: the claim stated after Algorithm 1 (with two seeds and one cross-edge
left, the cut edge is the longest one), its general form for alpha = 0 (the
two clusters are the components of the minimum spanning tree with the
heaviest edge on the tree path between the seeds removed), and the purpose of
the smoothing (alpha = 1 evens out the cluster populations).
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, dijkstra, minimum_spanning_tree


@pytest.fixture(scope="module")
def rn():
    from paper_1607_07696_amd import rn
    rn.load_library()
    return rn


def chain(rg, weights):
    n = len(weights) + 1
    return rg.from_edges(n, np.arange(n - 1), np.arange(1, n), np.asarray(weights), symmetric=True)


def test_chain_cut_at_heaviest_edge(rn, rg):
    rng = np.random.default_rng(0)
    for n in (3, 5, 17, 64):
        w = rng.permutation(np.arange(1, n)) * 10 + 5       # distinct weights
        g = chain(rg, w)
        part, _ = rn.partition_host(g.row_ptr, g.col, g.w, alpha=0.0, max_leaf=n - 1)
        cut = int(np.argmax(w))                                 # edge (cut, cut+1)
        assert len(set(part[: cut + 1])) == 1 and len(set(part[cut + 1:])) == 1
        assert part[cut] != part[cut + 1]


def _double_sweep(m):
    def far(s):
        d = dijkstra(m, directed=False, indices=s)
        d[np.isinf(d)] = -1
        return int(np.flatnonzero(d == d.max())[0])
    a = far(0)
    return a, far(a)


def test_alpha0_matches_mst_split(rn, rg):
    rng = np.random.default_rng(1)
    checked = 0
    for trial in range(200):
        n = int(rng.integers(4, 40))
        m_edges = int(rng.integers(n - 1, 3 * n))
        # random connected graph: a random spanning tree plus extra edges, distinct weights
        a = list(range(1, n))
        b = [int(rng.integers(0, i)) for i in range(1, n)]
        extra = rng.integers(0, n, size=(m_edges, 2))
        a += extra[:, 0].tolist()
        b += extra[:, 1].tolist()
        a, b = np.array(a), np.array(b)
        keep = a != b
        a, b = a[keep], b[keep]
        key = np.minimum(a, b) * n + np.maximum(a, b)
        _, first = np.unique(key, return_index=True)
        a, b = a[first], b[first]
        w = rng.permutation(len(a)) + 1
        g = rg.from_edges(n, a, b, w, symmetric=True)
        m = sp.csr_matrix((g.w.astype(float), g.col, g.row_ptr), shape=(n, n))
        s1, s2 = _double_sweep(m)
        if s1 == s2:
            continue
        mst = minimum_spanning_tree(m)
        mst = mst + mst.T
        # heaviest edge on the tree path s1 -> s2
        _, pred = dijkstra(mst, directed=False, indices=s1, return_predecessors=True)
        x, best, cut = s2, -1, None
        while x != s1:
            p = pred[x]
            if mst[p, x] > best:
                best, cut = mst[p, x], (p, x)
            x = p
        mst = mst.tolil()
        mst[cut[0], cut[1]] = 0
        mst[cut[1], cut[0]] = 0
        _, lab = connected_components(mst.tocsr(), directed=False)
        part, _ = rn.partition_host(g.row_ptr, g.col, g.w, alpha=0.0, max_leaf=n - 1)
        same = lab[:, None] == lab[None, :]
        assert np.array_equal(same, part[:, None] == part[None, :]), trial
        checked += 1
    assert checked > 150


def test_smoothing_evens_populations(rn, rg):
    n = 100
    w = np.arange(1, n)              # increasing weights: alpha = 0 cuts off one end vertex
    g = chain(rg, w)
    p0, _ = rn.partition_host(g.row_ptr, g.col, g.w, alpha=0.0, max_leaf=n - 1)
    p1, _ = rn.partition_host(g.row_ptr, g.col, g.w, alpha=1.0, max_leaf=n - 1)
    s0 = np.bincount(p0)
    s1 = np.bincount(p1)
    assert sorted(s0.tolist()) == [1, n - 1]
    assert s1.min() >= n // 5
    road = rg.road_graph(96, 0)
    sizes = {}
    for alpha in (0.0, 1.0):
        part, _ = rn.partition_host(road.row_ptr, road.col, road.w, alpha=alpha, max_leaf=512)
        sizes[alpha] = np.bincount(part)
    assert sizes[1.0].min() > sizes[0.0].min()
    assert len(sizes[1.0]) < len(sizes[0.0])


def test_partition_output_structure(rn, rg):
    g = rg.road_graph(64, 0)
    for alpha, leaf in ((0.0, 64), (0.5, 100), (1.0, 1), (1.0, 10 ** 6)):
        part, order = rn.partition_host(g.row_ptr, g.col, g.w, alpha=alpha, max_leaf=leaf)
        assert np.array_equal(np.sort(order), np.arange(g.V))
        assert np.bincount(part).max() <= leaf
        seq = part[order]
        assert np.all(np.diff(seq) >= 0)              # leaves contiguous, numbered in order
        assert seq[0] == 0 and np.all(np.diff(np.unique(seq)) == 1)
        p2, o2 = rn.partition_host(g.row_ptr, g.col, g.w, alpha=alpha, max_leaf=leaf)
        assert np.array_equal(part, p2) and np.array_equal(order, o2)


def test_disconnected_and_directed_inputs(rn, rg):
    g = rg.road_graph(12, 2, p_drop=0.5, keep_lcc=False)
    part, order = rn.partition_host(g.row_ptr, g.col, g.w, alpha=0.0, max_leaf=8)
    assert np.array_equal(np.sort(order), np.arange(g.V))
    assert np.bincount(part).max() <= 8
    d = rg.random_digraph(50, 120, 3, zero_frac=0.2)
    part, order = rn.partition_host(d.row_ptr, d.col, d.w, alpha=0.3, max_leaf=5)
    assert np.array_equal(np.sort(order), np.arange(50))
    assert np.bincount(part).max() <= 5
