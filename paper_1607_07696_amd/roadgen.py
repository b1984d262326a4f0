"""Seeded synthetic inputs: road-like graphs in CSR form and query node sets.

This module only *generates inputs*. It holds none of the join's arithmetic
(no shortest paths, no pair selection), so that the CPU oracle and the HIP path
can both be fed from it without sharing any of the method's code.

The paper evaluates on two real road networks (NA and SF, Section 5.1) that are
not available here; the graphs below stand in for them: sparse, near-planar,
average degree about 3.4, positive integer weights proportional to Euclidean
edge length.

Generator recipe (all draws from ``numpy.random.default_rng(seed)``, in this
order):

1. jitter ``U(-0.3, 0.3)`` for x then y of every grid node (row-major);
2. ``drop='edge'``: one ``U[0,1)`` per horizontal edge (i,j)-(i,j+1), then per
   vertical edge (i,j)-(i+1,j); the edge is kept iff the draw is ``>= p_drop``.
   ``drop='node'``: one draw per node instead, an edge is kept iff both ends are;
3. one draw per unit cell for the diagonal (i,j)-(i+1,j+1), then one per cell for
   (i,j+1)-(i+1,j); the diagonal is added iff the draw is ``< p_diag``;
4. one factor ``U(1.0, 1.5)`` per kept undirected edge (horizontal, vertical,
   diagonal-1, diagonal-2 order), so both arcs of an edge share one weight;
   ``w = floor(100 * |xy_a - xy_b| * factor + 0.5)`` computed in float64.

Only the largest connected component is kept (ties go to the component holding
the lowest node id) and it is renumbered in row-major order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

__all__ = [
    "Graph", "road_graph", "full_lattice", "random_digraph", "from_edges",
    "sample_disjoint", "sample_clustered", "batched_instances", "serving_stream",
]


@dataclass
class Graph:
    """A directed CSR graph with uint32 arc weights.

    ``row_ptr[x]..row_ptr[x+1]`` index the out-arcs of ``x``; arc ``a`` goes to
    ``col[a]`` with weight ``w[a]``.  Undirected inputs store each edge as two
    arcs of equal weight.
    """
    row_ptr: np.ndarray              # int32 [V+1]
    col: np.ndarray                  # int32 [A]
    w: np.ndarray                    # uint32 [A]
    xy: np.ndarray | None = None     # float32 [V,2] (optional)
    side: int = 0                    # grid side (0 if not a grid graph)
    cell: np.ndarray | None = field(default=None, repr=False)  # int32 [side*side] -> vertex id or -1

    @property
    def V(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def A(self) -> int:
        return int(self.col.shape[0])

    def outdeg(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def from_edges(V: int, src, dst, w, *, symmetric: bool, xy=None, side=0, cell=None) -> Graph:
    """Build a CSR from an arc (or edge, if ``symmetric``) list; arcs sorted by (src, dst)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w, dtype=np.uint32)
    if symmetric:
        src, dst, w = (np.concatenate([src, dst]), np.concatenate([dst, src]),
                       np.concatenate([w, w]))
    order = np.lexsort((dst, src))
    src, dst, w = src[order], dst[order], w[order]
    row_ptr = np.zeros(V + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=V), out=row_ptr[1:])
    return Graph(row_ptr.astype(np.int32), dst.astype(np.int32), w, xy, side, cell)


def _round_half_up(x: np.ndarray) -> np.ndarray:
    return np.floor(x + 0.5)


def road_graph(side: int, seed: int = 0, *, p_drop: float = 0.2, p_diag: float = 0.05,
               drop: str = "edge", keep_lcc: bool = True) -> Graph:
    """Synthetic road-like graph on a ``side`` x ``side`` grid (recipe in the module docstring)."""
    if drop not in ("edge", "node"):
        raise ValueError("drop must be 'edge' or 'node'")
    n = int(side)
    rng = np.random.default_rng(seed)
    ii, jj = np.divmod(np.arange(n * n, dtype=np.int64), n)
    xy = np.stack([jj, ii], axis=1).astype(np.float64) + rng.uniform(-0.3, 0.3, size=(n * n, 2))
    node_id = lambda i, j: i * n + j  # noqa: E731

    hi, hj = np.divmod(np.arange(n * (n - 1), dtype=np.int64), n - 1)
    h_a, h_b = node_id(hi, hj), node_id(hi, hj + 1)
    vi, vj = np.divmod(np.arange((n - 1) * n, dtype=np.int64), n)
    v_a, v_b = node_id(vi, vj), node_id(vi + 1, vj)
    if drop == "edge":
        h_keep = rng.random(h_a.shape[0]) >= p_drop
        v_keep = rng.random(v_a.shape[0]) >= p_drop
        node_keep = np.ones(n * n, dtype=bool)
    else:
        node_keep = rng.random(n * n) >= p_drop
        h_keep = node_keep[h_a] & node_keep[h_b]
        v_keep = node_keep[v_a] & node_keep[v_b]
    ci, cj = np.divmod(np.arange((n - 1) * (n - 1), dtype=np.int64), n - 1)
    d1_a, d1_b = node_id(ci, cj), node_id(ci + 1, cj + 1)
    d2_a, d2_b = node_id(ci, cj + 1), node_id(ci + 1, cj)
    d1_keep = rng.random(d1_a.shape[0]) < p_diag
    d2_keep = rng.random(d2_a.shape[0]) < p_diag
    if drop == "node":
        d1_keep &= node_keep[d1_a] & node_keep[d1_b]
        d2_keep &= node_keep[d2_a] & node_keep[d2_b]

    ea = np.concatenate([h_a[h_keep], v_a[v_keep], d1_a[d1_keep], d2_a[d2_keep]])
    eb = np.concatenate([h_b[h_keep], v_b[v_keep], d1_b[d1_keep], d2_b[d2_keep]])
    factor = rng.uniform(1.0, 1.5, size=ea.shape[0])
    length = np.hypot(xy[ea, 0] - xy[eb, 0], xy[ea, 1] - xy[eb, 1])
    w = _round_half_up(100.0 * length * factor).astype(np.uint32)

    present = node_keep.copy()
    if keep_lcc:
        adj = sp.coo_matrix((np.ones(ea.shape[0], dtype=np.int8), (ea, eb)), shape=(n * n, n * n))
        _, labels = connected_components(adj, directed=False)
        labels = np.where(node_keep, labels, -1)
        valid = labels >= 0
        sizes = np.bincount(labels[valid])
        # first occurrence of each label in id order is the component's lowest id
        lab_u, first = np.unique(labels[valid], return_index=True)
        min_id = np.flatnonzero(valid)[first]
        best = max(range(lab_u.shape[0]), key=lambda t: (sizes[lab_u[t]], -min_id[t]))
        present = labels == lab_u[best]
    new_id = np.full(n * n, -1, dtype=np.int64)
    new_id[present] = np.arange(int(present.sum()))
    keep_e = present[ea] & present[eb]
    V = int(present.sum())
    return from_edges(V, new_id[ea[keep_e]], new_id[eb[keep_e]], w[keep_e], symmetric=True,
                      xy=xy[present].astype(np.float32), side=n,
                      cell=new_id.astype(np.int32))


def full_lattice(side: int, weight: int) -> Graph:
    """Full ``side`` x ``side`` 4-neighbour lattice, every edge of weight ``weight``.

    Its shortest-path distances have the closed form
    ``weight * (|i1 - i2| + |j1 - j2|)`` for nodes (i1, j1), (i2, j2).
    """
    n = int(side)
    hi, hj = np.divmod(np.arange(n * (n - 1), dtype=np.int64), n - 1)
    vi, vj = np.divmod(np.arange((n - 1) * n, dtype=np.int64), n)
    ea = np.concatenate([hi * n + hj, vi * n + vj])
    eb = np.concatenate([hi * n + hj + 1, (vi + 1) * n + vj])
    ii, jj = np.divmod(np.arange(n * n), n)
    xy = np.stack([jj, ii], axis=1).astype(np.float32)
    return from_edges(n * n, ea, eb, np.full(ea.shape[0], weight, dtype=np.uint32),
                      symmetric=True, xy=xy, side=n, cell=np.arange(n * n, dtype=np.int32))


def random_digraph(V: int, A: int, seed: int, *, wmin: int = 1, wmax: int = 100,
                   zero_frac: float = 0.0, self_loops: bool = True) -> Graph:
    """Random directed multigraph: ``A`` arcs with uniform endpoints and weights.

    ``zero_frac`` of the arcs get weight 0; self-loops and parallel arcs are
    allowed unless ``self_loops`` is False.
    """
    rng = np.random.default_rng(seed)
    src = rng.integers(0, V, size=A)
    dst = rng.integers(0, V, size=A)
    if not self_loops:
        dst = np.where(dst == src, (dst + 1) % V, dst)
    w = rng.integers(wmin, wmax + 1, size=A)
    if zero_frac > 0:
        w = np.where(rng.random(A) < zero_frac, 0, w)
    return from_edges(V, src, dst, w, symmetric=False)


def sample_disjoint(V: int, nR: int, nS: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Disjoint uniform samples: ``nR + nS`` distinct nodes, the first ``nR`` form R."""
    if nR + nS > V:
        raise ValueError("nR + nS exceeds V")
    rng = np.random.default_rng(seed)
    idx = rng.choice(V, size=nR + nS, replace=False).astype(np.int32)
    return idx[:nR].copy(), idx[nR:].copy()


def sample_clustered(g: Graph, nR: int, nS: int, seed: int, *, n_clusters: int = 32,
                     sigma: float = 20.0, frac_uniform: float = 0.5
                     ) -> tuple[np.ndarray, np.ndarray]:
    """Disjoint R, S: ``frac_uniform`` of each drawn uniformly, the rest around shared centres.

    Centres are uniform in the grid and shared by R and S.  A clustered point is
    ``centre + N(0, sigma^2)`` per axis rounded to a grid cell; it is redrawn if the
    cell is outside the grid, not in the graph, or already taken.
    """
    if g.cell is None or g.side <= 0:
        raise ValueError("clustered sampling needs a grid graph")
    if nR + nS > g.V:
        raise ValueError("nR + nS exceeds V")
    n = g.side
    rng = np.random.default_rng(seed)
    nRu, nSu = int(round(nR * frac_uniform)), int(round(nS * frac_uniform))
    uni = rng.choice(g.V, size=nRu + nSu, replace=False).astype(np.int64)
    taken = np.zeros(g.V, dtype=bool)
    taken[uni] = True
    centres = rng.uniform(0.0, n - 1, size=(n_clusters, 2))
    need = (nR - nRu) + (nS - nSu)
    got: list[np.ndarray] = []
    have = 0
    while have < need:
        m = max(1024, 2 * (need - have))
        c = rng.integers(0, n_clusters, size=m)
        p = np.floor(centres[c] + rng.normal(0.0, sigma, size=(m, 2)) + 0.5).astype(np.int64)
        ok = (p[:, 0] >= 0) & (p[:, 0] < n) & (p[:, 1] >= 0) & (p[:, 1] < n)
        vid = np.full(m, -1, dtype=np.int64)
        vid[ok] = g.cell[p[ok, 1] * n + p[ok, 0]]
        vid = vid[vid >= 0]
        # keep first occurrences in draw order, skipping taken cells
        _, first = np.unique(vid, return_index=True)
        vid = vid[np.sort(first)]
        vid = vid[~taken[vid]][: need - have]
        taken[vid] = True
        got.append(vid)
        have += vid.shape[0]
    clus = np.concatenate(got) if got else np.zeros(0, dtype=np.int64)
    R = np.concatenate([uni[:nRu], clus[: nR - nRu]]).astype(np.int32)
    S = np.concatenate([uni[nRu:], clus[nR - nRu:]]).astype(np.int32)
    return R, S


def _log_uniform_int(rng, lo: int, hi: int, size=None):
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))).astype(np.int64)


@dataclass
class Instance:
    graph: Graph
    R: np.ndarray
    S: np.ndarray
    theta: int
    k: int          # 0 for a theta-join, else k-closest pairs


def batched_instances(count: int = 128, base_seed: int = 1000) -> list[Instance]:
    """Independent graph + join instances; instance ``i`` is drawn from seed ``base_seed + i``.

    Side log-uniform in [32, 512]; |R|, |S| log-uniform in [16, 4096] (clamped so
    they fit the graph); theta uniform in [500, 5000]; odd instances ask for k
    closest pairs with k log-uniform in [1, 1024].
    """
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        side = int(_log_uniform_int(rng, 32, 512))
        nR = int(_log_uniform_int(rng, 16, 4096))
        nS = int(_log_uniform_int(rng, 16, 4096))
        theta = int(rng.integers(500, 5001))
        k = int(_log_uniform_int(rng, 1, 1024)) if (i % 2 == 1) else 0
        g = road_graph(side, seed=base_seed + i)
        nR = min(nR, g.V // 2)
        nS = min(nS, g.V - nR)
        R, S = sample_disjoint(g.V, nR, nS, seed=base_seed + i)
        out.append(Instance(g, R, S, theta, k))
    return out


@dataclass
class Request:
    arrival_s: float
    R: np.ndarray
    S: np.ndarray
    theta: int
    k: int          # 0 for a theta-join


def shuffle_ids(g: Graph, seed: int) -> tuple[Graph, np.ndarray]:
    """The same graph with its vertex ids permuted at random (no locality left
    in the numbering); returns it and perm (old id -> new id)."""
    perm = np.random.default_rng(seed).permutation(g.V).astype(np.int32)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.V, dtype=np.int32)
    deg = np.diff(g.row_ptr)[inv]
    row = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    col = np.empty(g.A, np.int32)
    w = np.empty(g.A, np.uint32)
    for xn in range(g.V):
        b, e = g.row_ptr[inv[xn]], g.row_ptr[inv[xn] + 1]
        col[row[xn]:row[xn + 1]] = perm[g.col[b:e]]
        w[row[xn]:row[xn + 1]] = g.w[b:e]
    return Graph(row, col, w), perm


def serving_stream(g: Graph, count: int, rate_hz: float, seed: int = 5, *,
                   kcp_frac: float = 0.4) -> list[Request]:
    """Poisson request stream: ``kcp_frac`` k-closest-pairs requests, the rest theta-joins.

    |R|, |S| log-uniform in [64, 32768]; theta uniform in [500, 8000]; k
    log-uniform in [1, 4096].
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=count))
    reqs = []
    for i in range(count):
        nR = int(_log_uniform_int(rng, 64, 32768))
        nS = int(_log_uniform_int(rng, 64, 32768))
        is_kcp = rng.random() < kcp_frac
        theta = int(rng.integers(500, 8001))
        k = int(_log_uniform_int(rng, 1, 4096)) if is_kcp else 0
        idx = rng.choice(g.V, size=nR + nS, replace=False).astype(np.int32)
        reqs.append(Request(float(t[i]), idx[:nR].copy(), idx[nR:].copy(), theta, k))
    return reqs
