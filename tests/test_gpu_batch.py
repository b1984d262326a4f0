"""GPU parity of the batched form: many queries, on one or many graphs, per call.

Every query's segment of a batch must equal, bit for bit, the oracle's answer
for that query alone (tolerance 0): the theta-join list, or the first k pairs
of the (dist, u, v) order within theta.
"""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MAX_DIST = 0xFFFFFFFE


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def rnmod(torch_cuda):
    from paper_1607_07696_amd import rn
    rn.load_library()
    return rn


@pytest.fixture(scope="module")
def instances(rg):
    return rg.batched_instances(128)


def oracle_answer(orc, g, R, S, theta, k):
    if k == 0:
        return orc.dist_join(g, R, S, theta).pairs
    if theta >= MAX_DIST:
        return orc.kcp_join(g, R, S, k)
    return orc.dist_join(g, R, S, theta).pairs[:k]      # k closest pairs within theta


def assert_same(got, want, what=""):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    assert np.array_equal(got, want), what


def spec(inst, graph):
    # the batched workload's k-closest-pairs instances are unbounded
    return {"R": inst.R, "S": inst.S, "graph": graph, "k": inst.k,
            "theta": inst.theta if inst.k == 0 else MAX_DIST}


def check_batch(rnmod, orc, out, off, status, cases):
    assert not status.any()
    got = rnmod.split_batch(out, off)
    for i, (g, R, S, theta, k) in enumerate(cases):
        assert_same(got[i], oracle_answer(orc, g, R, S, theta, k), f"query {i}")


def test_config4_128_instances_one_call(rnmod, orc, instances):
    net = rnmod.RoadNetwork.from_graphs([x.graph for x in instances])
    assert net.num_graphs == 128
    specs = [spec(x, i) for i, x in enumerate(instances)]
    out, off, status = net.join_batch(specs)
    cases = [(x.graph, x.R, x.S, s["theta"], x.k) for x, s in zip(instances, specs)]
    check_batch(rnmod, orc, out, off, status, cases)


def test_batch_with_partition_and_autotune(rnmod, orc, instances):
    sub = instances[:40]
    net = rnmod.RoadNetwork.from_graphs([x.graph for x in sub])
    net.partition(1.0, 128)
    q, keep = net.make_queries([spec(x, i) for i, x in enumerate(sub)])
    net.autotune(q, sample=64)
    assert all(8 <= q[i].hash_log2 <= 14 or q[i].hash_log2 == rnmod.RN_TABLE_GLOBAL for i in range(len(sub)))
    out, off, status = net.join_batch(q)
    cases = [(x.graph, x.R, x.S, x.theta if x.k == 0 else MAX_DIST, x.k) for x in sub]
    check_batch(rnmod, orc, out, off, status, cases)


def test_many_queries_on_one_graph_match_single_calls(rnmod, orc, rg):
    g = rg.road_graph(160, 2)
    net = rnmod.RoadNetwork.from_graph(g)
    cases = []
    for i in range(12):
        R, S = rg.sample_disjoint(g.V, 50 + 40 * i, 300 - 20 * i, 100 + i)
        theta = [0, 700, 1500, 2500, 4000, MAX_DIST][i % 6]
        k = [0, 0, 5, 0, 300, 40][i % 6] if theta != MAX_DIST else 77
        cases.append((g, R, S, theta, k))
    specs = [{"R": R, "S": S, "theta": t, "k": k} for _, R, S, t, k in cases]
    out, off, status = net.join_batch(specs)
    check_batch(rnmod, orc, out, off, status, cases)
    # the single-query calls give the same lists
    got = rnmod.split_batch(out, off)
    for i, (_, R, S, theta, k) in enumerate(cases):
        if k == 0:
            assert_same(rnmod.pairs_to_numpy(net.dist_join(R, S, theta)), got[i])
        elif theta == MAX_DIST:
            assert_same(rnmod.pairs_to_numpy(net.kcp_join(R, S, k)), got[i])


def test_per_query_tuning_and_tiers(rnmod, orc, rg):
    g = rg.road_graph(96, 5)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 80, 400, 31)
    specs, cases = [], []
    for i, (hb, delta) in enumerate([(8, 0), (9, 46), (10, None), (12, 0), (13, 500), (14, 1), (0, None)]):
        theta = 6000 if i % 2 == 0 else 2500
        k = 0 if i < 5 else 50
        specs.append({"R": R, "S": S, "theta": theta, "k": k, "hash_log2": hb, "delta": delta})
        cases.append((g, R, S, theta, k))
    # searches in the global tier from the start, beside the on-chip groups
    # (theta-joins and k-closest pairs together: they share the tier's slots)
    for theta, k in ((6000, 0), (2500, 50), (MAX_DIST, 300), (4000, 0)):
        specs.append({"R": R, "S": S, "theta": theta, "k": k, "hash_log2": rnmod.RN_TABLE_GLOBAL})
        cases.append((g, R, S, theta, k))
    out, off, status = net.join_batch(specs)
    check_batch(rnmod, orc, out, off, status, cases)
    # and in a captured plan, replayed
    q, keep = net.make_queries(specs)
    plan = net.plan(q)
    for _ in range(2):
        out, off, status = plan.run()
        check_batch(rnmod, orc, out, off, status, cases)
    plan.close()


def test_invalid_query_gets_empty_segment(rnmod, orc, rg):
    g = rg.road_graph(64, 0)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 64, 64, 1)
    Rbad = R.copy()
    Rbad[3] = R[5]
    specs = [{"R": R, "S": S, "theta": 1500}, {"R": Rbad, "S": S, "theta": 1500},
             {"R": R, "S": S, "k": 16}]
    out, off, status = net.join_batch(specs, check=False)
    assert list(status) == [rnmod.RN_OK, rnmod.RN_ERR_ARG, rnmod.RN_OK]
    got = rnmod.split_batch(out, off)
    assert_same(got[0], orc.dist_join(g, R, S, 1500).pairs)
    assert got[1].shape[0] == 0
    assert_same(got[2], orc.kcp_join(g, R, S, 16))
    with pytest.raises(rnmod.RnError) as ei:
        net.join_batch(specs)
    assert ei.value.status == rnmod.RN_ERR_ARG


def test_host_side_query_errors(rnmod, rg, torch_cuda):
    g = rg.road_graph(64, 0)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 10, 10, 2)
    for bad in ({"graph": 1}, {"k": -1}, {"hash_log2": 7}, {"k": (1 << 24) + 1}):
        sp = {"R": R, "S": S, "theta": 100, **bad}
        with pytest.raises(rnmod.RnError) as ei:
            net.join_batch([{"R": R, "S": S, "theta": 100}, sp])
        assert ei.value.status == rnmod.RN_ERR_ARG


def test_batch_capacity_two_call_convention(rnmod, orc, rg, torch_cuda):
    torch = torch_cuda
    g = rg.road_graph(64, 0)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 64, 64, 1)
    q, keep = net.make_queries([{"R": R, "S": S, "theta": 1500}, {"R": R, "S": S, "k": 16}])
    want0 = orc.dist_join(g, R, S, 1500).pairs
    lib = rnmod.load_library()
    off = np.zeros(3, dtype=np.int64)
    small = torch.zeros((7, 3), dtype=torch.int32, device="cuda")
    st = lib.rn_join_batch(net._h, q, 2, C.c_void_p(small.data_ptr()), 7,
                           off.ctypes.data_as(C.POINTER(C.c_int64)), None, None)
    assert st == rnmod.RN_ERR_CAPACITY
    assert off[1] == len(want0) and off[2] == len(want0) + 16
    assert torch.count_nonzero(small).item() == 0
    big = torch.zeros((int(off[2]), 3), dtype=torch.int32, device="cuda")
    st = lib.rn_join_batch(net._h, q, 2, C.c_void_p(big.data_ptr()), int(off[2]),
                           off.ctypes.data_as(C.POINTER(C.c_int64)), None, None)
    assert st == rnmod.RN_OK
    a = rnmod.pairs_to_numpy(big)
    assert_same(a[: off[1]], want0)
    assert_same(a[off[1]:], orc.kcp_join(g, R, S, 16))


def test_plan_replays_match_eager(rnmod, orc, rg, torch_cuda, instances):
    torch = torch_cuda
    sub = instances[:24]
    net = rnmod.RoadNetwork.from_graphs([x.graph for x in sub])
    q, keep = net.make_queries([spec(x, i) for i, x in enumerate(sub)])
    eager_out, eager_off, _ = net.join_batch(q)
    eager = rnmod.pairs_to_numpy(eager_out)
    plan = net.plan(q)
    for rep in range(4):
        out, off, status = plan.run()
        assert not status.any()
        assert np.array_equal(off, eager_off), rep
        assert_same(rnmod.pairs_to_numpy(out), eager, f"replay {rep}")
        # eager work and a synchronisation between replays
        net.join_batch([spec(sub[1], 1)])
        torch.cuda.synchronize()
    cases = [(x.graph, x.R, x.S, x.theta if x.k == 0 else MAX_DIST, x.k) for x in sub]
    check_batch(rnmod, orc, out, off, status, cases)
    # new contents of R in place (same size): the replay follows them
    i0 = next(i for i, x in enumerate(sub) if x.k == 0)
    x = sub[i0]
    R2, S2 = rg.sample_disjoint(x.graph.V, len(x.R), len(x.S), 999)
    keep[2 * i0].copy_(torch.as_tensor(R2))
    keep[2 * i0 + 1].copy_(torch.as_tensor(S2))
    out, off, status = plan.run()
    got = rnmod.split_batch(out, off)
    assert_same(got[i0], orc.dist_join(x.graph, R2, S2, x.theta).pairs)
    plan.close()


def test_plan_regrows_its_record_buffer(rnmod, orc, rg, torch_cuda):
    torch = torch_cuda
    # two disconnected copies of one road graph
    a = rg.road_graph(100, 3)
    V, A = a.V, a.A
    g = rg.Graph(np.concatenate([a.row_ptr, a.row_ptr[1:] + A]).astype(np.int32),
                 np.concatenate([a.col, a.col + V]).astype(np.int32), np.concatenate([a.w, a.w]))
    R, S = rg.sample_disjoint(V, 500, 3000, 41)
    Rt = torch.as_tensor(R + V, device="cuda")          # R in the other copy: no pair at all
    St = torch.as_tensor(S, device="cuda")
    net = rnmod.RoadNetwork.from_graph(g)
    q, keep = net.make_queries([{"R": Rt, "S": St, "theta": MAX_DIST}])
    plan = net.plan(q, cap=len(R) * len(S))
    out, off, _ = plan.run()
    assert off[1] == 0
    # R moved next to S: 1.5M records, more than the plan was sized for, so
    # the run re-sizes, re-runs and re-captures
    Rt.copy_(torch.as_tensor(R, device="cuda"))
    want = orc.dist_join(g, R, S, MAX_DIST).pairs
    assert len(want) == len(R) * len(S)
    for _ in range(2):
        out, off, _ = plan.run()
        assert_same(rnmod.pairs_to_numpy(out), want)
    plan.close()


def test_kcp_within_theta(rnmod, orc, rg):
    g = rg.road_graph(128, 7)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 300, 300, 51)
    specs, cases = [], []
    for theta, k in ((800, 10), (800, 100000), (1500, 500), (0, 3), (3000, 1)):
        specs.append({"R": R, "S": S, "theta": theta, "k": k})
        cases.append((g, R, S, theta, k))
    out, off, status = net.join_batch(specs)
    check_batch(rnmod, orc, out, off, status, cases)


@pytest.mark.parametrize("sort", ["bucket", "radix"])
def test_more_than_1024_queries_in_one_call(rnmod, orc, rg, sort):
    """2 100 small queries in one call: the per-query layout (kept counts,
    segment starts, output offsets) is scanned 1 024 queries at a time with
    totals carried between blocks, and the last block is ragged.  A random
    digraph with weights 1..40 gives pairs at small theta.  "bucket":
    theta-joins only with sum(theta + 1) <= 65 536 on a graph of varied
    weights, so the (query, dist) bucket sort runs; "radix": every seventh
    query asks for the k closest pairs, which sends the call to the radix
    sort."""
    g = rg.random_digraph(300, 1500, 21, wmin=1, wmax=40)
    net = rnmod.RoadNetwork.from_graph(g)
    rng = np.random.default_rng(77)
    cases = []
    for i in range(2100):
        R, S = rg.sample_disjoint(g.V, int(rng.integers(1, 11)), int(rng.integers(1, 11)), 5000 + i)
        if sort == "bucket":
            theta, k = i % 40, 0
        elif i % 7 == 3:
            theta, k = MAX_DIST, int(rng.integers(1, 9))
        else:
            theta, k = int(rng.integers(0, 61)), 0
        cases.append((g, R, S, theta, k))
    if sort == "bucket":
        assert sum(t + 1 for _, _, _, t, _ in cases) <= 65536
    specs = [{"R": R, "S": S, "theta": t, "k": k} for _, R, S, t, k in cases]
    out, off, status = net.join_batch(specs)
    assert int(off[-1]) > 1000
    check_batch(rnmod, orc, out, off, status, cases)


def test_config4_autotuned_plan_all_instances(rnmod, orc, instances, torch_cuda):
    # the batched workload's headline form: all 128 instances autotuned (the
    # benchmark's sample of 256 sources per query), captured as one plan and
    # replayed, every replay checked against the oracle, with eager work and a
    # synchronisation between replays
    torch = torch_cuda
    net = rnmod.RoadNetwork.from_graphs([x.graph for x in instances])
    q, keep = net.make_queries([spec(x, i) for i, x in enumerate(instances)])
    net.autotune(q, sample=256)
    plan = net.plan(q)
    cases = [(x.graph, x.R, x.S, x.theta if x.k == 0 else MAX_DIST, x.k) for x in instances]
    wants = [oracle_answer(orc, *c) for c in cases]
    for rep in range(3):
        out, off, status = plan.run()
        assert not status.any()
        got = rnmod.split_batch(out, off)
        for i, w in enumerate(wants):
            assert_same(got[i], w, f"replay {rep}, instance {i}")
        net.join_batch([spec(instances[3], 3)])
        torch.cuda.synchronize()
    plan.close()
