"""GPU parity of joins over objects on edges (Section 1): objects inserted into
their edges as vertices (rn_objects_graph), joined on the device, against the
oracle's object join (tolerance 0)."""
import numpy as np
import pytest

from test_objects import random_objects

pytestmark = pytest.mark.gpu

MAX_DIST = 0xFFFFFFFE


@pytest.fixture(scope="module")
def rnmod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1607_07696_amd import rn
    rn.load_library()
    return rn


def to_objects(pairs, V, nR):
    # device pairs name object i as vertex V + i; S objects follow the R ones
    out = np.zeros(len(pairs), dtype=pairs.dtype)
    out["u"] = pairs["u"] - V
    out["v"] = pairs["v"] - V - nR
    out["dist"] = pairs["dist"]
    return out


@pytest.mark.parametrize("side,seed,nR,nS", [(96, 3, 300, 400), (40, 8, 60, 50)])
def test_object_joins_match_oracle(rnmod, orc, rg, side, seed, nR, nS):
    g = rg.road_graph(side, seed)
    rng = np.random.default_rng(seed)
    Ra, Ro = random_objects(g, nR, rng)
    Sa, So = random_objects(g, nS, rng, share=Ra)
    net = rnmod.RoadNetwork.from_graph(g)
    onet = net.with_objects(np.concatenate([Ra, Sa]), np.concatenate([Ro, So]))
    assert onet.V == g.V + nR + nS
    Rv = np.arange(g.V, g.V + nR, dtype=np.int32)
    Sv = np.arange(g.V + nR, g.V + nR + nS, dtype=np.int32)
    for theta in (0, 300, 1500, 4000):
        got = to_objects(rnmod.pairs_to_numpy(onet.dist_join(Rv, Sv, theta)), g.V, nR)
        want = orc.object_join(g, Ra, Ro, Sa, So, theta)
        assert got.shape == want.shape and np.array_equal(got, want), theta
    allp = orc.object_join(g, Ra, Ro, Sa, So, MAX_DIST)
    for k in (1, 50, 2000):
        got = to_objects(rnmod.pairs_to_numpy(onet.kcp_join(Rv, Sv, k)), g.V, nR)
        assert np.array_equal(got, allp[:k]), k
    # the graph's own vertices keep their distances
    R, S = rg.sample_disjoint(g.V, 50, 50, seed + 1)
    a = rnmod.pairs_to_numpy(onet.dist_join(R, S, 2000))
    b = rnmod.pairs_to_numpy(net.dist_join(R, S, 2000))
    assert np.array_equal(a, b)


def test_objects_on_a_directed_multigraph(rnmod, orc, rg):
    # one-way arcs, parallel arcs and loops: objects on them move and are
    # reached in the arcs' direction only, two-way roads both ways
    g = rg.random_digraph(400, 1600, 5, wmin=0, wmax=60, zero_frac=0.05)
    rng = np.random.default_rng(9)
    Ra, Ro = random_objects(g, 80, rng)
    Sa, So = random_objects(g, 90, rng, share=Ra)
    net = rnmod.RoadNetwork.from_graph(g)
    onet = net.with_objects(np.concatenate([Ra, Sa]), np.concatenate([Ro, So]))
    Rv = np.arange(g.V, g.V + 80, dtype=np.int32)
    Sv = np.arange(g.V + 80, g.V + 170, dtype=np.int32)
    for theta in (0, 40, 150, MAX_DIST):
        got = to_objects(rnmod.pairs_to_numpy(onet.dist_join(Rv, Sv, theta)), g.V, 80)
        assert np.array_equal(got, orc.object_join(g, Ra, Ro, Sa, So, theta)), theta


def test_object_argument_errors(rnmod, rg):
    g = rg.road_graph(16, 0)
    net = rnmod.RoadNetwork.from_graph(g)
    for arcs, offs in (([g.A], [0]), ([-1], [0]), ([0], [int(g.w[0]) + 1])):
        with pytest.raises(rnmod.RnError) as ei:
            net.with_objects(arcs, offs)
        assert ei.value.status == rnmod.RN_ERR_ARG
