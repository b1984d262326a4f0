"""Seeded input generators: shapes, determinism and the stated recipe."""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


def _csr(g):
    return sp.csr_matrix((g.w.astype(np.float64), g.col, g.row_ptr), shape=(g.V, g.V))


def test_small_grid_sizes_and_determinism(rg):
    g = rg.road_graph(64, 0)
    g2 = rg.road_graph(64, 0)
    assert g.V == 4091 and g.A == 13768
    for a, b in ((g.row_ptr, g2.row_ptr), (g.col, g2.col), (g.w, g2.w)):
        assert np.array_equal(a, b)
    assert g.row_ptr.dtype == np.int32 and g.col.dtype == np.int32 and g.w.dtype == np.uint32
    assert not np.array_equal(rg.road_graph(64, 1).w[:100], g.w[:100])


def test_csr_is_symmetric_connected_and_simple(rg):
    g = rg.road_graph(64, 0)
    m = _csr(g)
    assert (m != m.T).nnz == 0                       # each edge stored twice, same weight
    assert connected_components(m, directed=False)[0] == 1   # only the LCC is kept
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    assert np.all(src != g.col)                      # no self-loops
    key = src.astype(np.int64) * g.V + g.col
    assert np.unique(key).shape[0] == g.A            # no parallel arcs
    assert np.all(np.diff(key) > 0)                  # arcs sorted by (src, dst)


def test_weights_follow_recipe(rg):
    g = rg.road_graph(64, 0)
    src = np.repeat(np.arange(g.V), np.diff(g.row_ptr))
    length = np.hypot(*(g.xy[src] - g.xy[g.col]).T.astype(np.float64))
    ratio = g.w / (100.0 * length)
    # factor in [1, 1.5] up to rounding of w and float32 coordinates
    assert ratio.min() > 1.0 - 0.6 / 40 and ratio.max() < 1.5 + 0.6 / 40
    assert g.w.min() >= 40                           # axis edges are at least 0.4 long
    deg = np.diff(g.row_ptr)
    assert deg.max() <= 8 and 3.2 < deg.mean() < 3.6


def test_node_drop_mode_is_smaller(rg):
    e = rg.road_graph(64, 0, drop="edge")
    n = rg.road_graph(64, 0, drop="node")
    assert n.V < e.V
    assert 0.7 * 64 * 64 < n.V < 0.85 * 64 * 64


def test_disjoint_samples(rg):
    R, S = rg.sample_disjoint(4091, 64, 64, 1)
    assert R.shape == (64,) and S.shape == (64,)
    assert len(set(R) | set(S)) == 128
    R2, _ = rg.sample_disjoint(4091, 64, 64, 1)
    assert np.array_equal(R, R2)


def test_clustered_samples(rg):
    g = rg.road_graph(128, 0)
    R, S = rg.sample_clustered(g, 1024, 1024, 3)
    assert len(set(R.tolist()) | set(S.tolist())) == 2048
    assert R.min() >= 0 and R.max() < g.V
    # clustered halves concentrate: their mean nearest-neighbour distance is smaller
    xy = g.xy
    def spread(ids):
        p = xy[ids]
        d = np.hypot(p[:, None, 0] - p[None, :, 0], p[:, None, 1] - p[None, :, 1])
        np.fill_diagonal(d, np.inf)
        return d.min(axis=1).mean()
    assert spread(R[512:]) < spread(R[:512])


def test_full_lattice_closed_form_shape(rg):
    g = rg.full_lattice(5, 7)
    assert g.V == 25 and g.A == 2 * 2 * 5 * 4
    assert np.all(g.w == 7)


def test_batched_instances_shapes(rg):
    inst = rg.batched_instances(count=4)
    assert len(inst) == 4
    for i, it in enumerate(inst):
        assert 32 * 32 * 0.5 < it.graph.V <= 512 * 512
        assert 16 <= len(it.R) <= 4096 and len(it.R) + len(it.S) <= it.graph.V
        assert 500 <= it.theta <= 5000
        assert (it.k > 0) == (i % 2 == 1)


def test_shuffle_ids_relabels_the_same_graph(rg, orc):
    g = rg.road_graph(48, 3)
    gs, perm = rg.shuffle_ids(g, 9)
    assert gs.V == g.V and gs.A == g.A and sorted(perm.tolist()) == list(range(g.V))
    R, S = rg.sample_disjoint(g.V, 40, 40, 10)
    a = orc.dist_join(g, R, S, 1500).pairs
    b = orc.dist_join(gs, perm[R], perm[S], 1500).pairs
    # the same pairs under the relabelling
    mapped = sorted(zip(a["dist"].tolist(), perm[a["u"]].tolist(), perm[a["v"]].tolist()))
    assert mapped == sorted(zip(b["dist"].tolist(), b["u"].tolist(), b["v"].tolist()))
