"""GPU theta-join parity: the HIP path against the CPU oracle, bit for bit.

Every result is an integer list sorted by (dist, u, v), so the comparison is
exact equality of the pair arrays (tolerance 0).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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
def g64(rg):
    return rg.road_graph(64, 0)


@pytest.fixture(scope="module")
def g1024(rg):
    return rg.road_graph(1024, 0)


def gpu_join(rnmod, net, R, S, theta):
    return rnmod.pairs_to_numpy(net.dist_join(R, S, theta))


def assert_same(got, want):
    assert got.shape == want.shape, (got.shape, want.shape)
    assert np.array_equal(got, want)


def test_config1_theta_join(rnmod, orc, rg, g64):
    net = rnmod.RoadNetwork.from_graph(g64)
    R, S = rg.sample_disjoint(g64.V, 64, 64, 1)
    want = orc.dist_join(g64, R, S, 1500).pairs
    assert len(want) > 100
    assert_same(gpu_join(rnmod, net, R, S, 1500), want)


def test_config2_theta_join_full_size(rnmod, orc, rg, g1024):
    net = rnmod.RoadNetwork.from_graph(g1024)
    R, S = rg.sample_disjoint(g1024.V, 8192, 8192, 2)
    ref = orc.dist_join(g1024, R, S, 3000)
    want = ref.pairs
    assert len(want) > 50000
    assert_same(gpu_join(rnmod, net, R, S, 3000), want)
    # second call on the same handle (buffers reused), with work counting on:
    # the GPU's settled (source, vertex) set has the oracle's size and arc total
    net.set_profiling(times=True, work=True)
    assert_same(gpu_join(rnmod, net, R, S, 3000), want)
    st = net.stats()
    assert st["settled"] == ref.settled and st["arcs"] == ref.arcs
    # the launch configuration the benchmark times: sources in partition
    # order (alpha 1, leaves of 256), the query captured once as a plan and
    # replayed; every replay equals the oracle
    net.set_profiling(times=False, work=False)
    net.partition(1.0, 256)
    q, keep = net.make_queries([{"R": R, "S": S, "theta": 3000}])
    plan = net.plan(q, cap=len(want) + 1024)
    for _ in range(3):
        out, off, status = plan.run()
        assert not status.any() and int(off[-1]) == len(want)
        assert_same(rnmod.pairs_to_numpy(out), want)
    plan.close()


@pytest.mark.parametrize("theta", [0, 1, 41, 700, 1500, 2999])
def test_thetas_small_graph(rnmod, orc, rg, g64, theta):
    net = rnmod.RoadNetwork.from_graph(g64)
    R, S = rg.sample_disjoint(g64.V, 300, 500, 7)
    assert_same(gpu_join(rnmod, net, R, S, theta), orc.dist_join(g64, R, S, theta).pairs)


@pytest.mark.parametrize("delta", [0, 1, 46, 150, 1000, 0xFFFFFFFE])
def test_bucket_width_never_changes_results(rnmod, orc, rg, g64, delta):
    net = rnmod.RoadNetwork.from_graph(g64)
    net.set_tuning(delta=delta)
    R, S = rg.sample_disjoint(g64.V, 128, 256, 8)
    assert_same(gpu_join(rnmod, net, R, S, 2500), orc.dist_join(g64, R, S, 2500).pairs)


@pytest.mark.parametrize("hash_log2", [8, 9, 10, 11, 12, 13, 14])
def test_table_tiers_and_reruns(rnmod, orc, rg, g64, hash_log2):
    net = rnmod.RoadNetwork.from_graph(g64)
    net.set_tuning(hash_log2=hash_log2)
    R, S = rg.sample_disjoint(g64.V, 64, 96, 9)
    for theta in (1500, 6000):
        assert_same(gpu_join(rnmod, net, R, S, theta), orc.dist_join(g64, R, S, theta).pairs)
    st = net.stats()
    if hash_log2 <= 10:
        assert st["retried"] > 0          # the small first table overflowed and was re-run


@pytest.mark.parametrize("hash_log2", [10, 11])
def test_wide_tables_for_distances_beyond_the_compact_word(rnmod, orc, rg, hash_log2):
    # theta above the largest distance a compact table of this size holds, so
    # the first tier is the wide table; the whole 20x20 graph fits it
    g = rg.road_graph(20, 3)
    g.w = (g.w * 64).astype(np.uint32)
    net = rnmod.RoadNetwork.from_graph(g)
    net.set_tuning(hash_log2=hash_log2)
    net.set_profiling(times=True, work=False)
    R, S = rg.sample_disjoint(g.V, 48, 200, 12)
    theta = 90000
    want = orc.dist_join(g, R, S, theta).pairs
    assert len(want) > 3000 and int(want["dist"].max()) > 16382
    assert_same(gpu_join(rnmod, net, R, S, theta), want)
    assert net.stats()["retried"] == 0


def test_whole_graph_ball(rnmod, orc, rg, g64):
    net = rnmod.RoadNetwork.from_graph(g64)
    R, S = rg.sample_disjoint(g64.V, 16, 2000, 10)
    theta = 0xFFFFFFFE
    assert_same(gpu_join(rnmod, net, R, S, theta), orc.dist_join(g64, R, S, theta).pairs)


def test_pending_sets_beyond_the_ring_go_to_the_next_tier(rnmod, orc, rg):
    # a hub of 300 spokes: the first step from the hub leaves 300 vertices
    # pending, more than the compact 2^11 search's ring holds, while the
    # 301 vertices fit its table; the search goes on to the next tier
    n = 300
    rng = np.random.default_rng(21)
    src = np.concatenate([np.zeros(n, dtype=np.int64), np.arange(1, n + 1)])
    dst = np.concatenate([np.arange(1, n + 1), np.roll(np.arange(1, n + 1), 1)])
    w = rng.integers(5, 40, size=2 * n)
    g = rg.from_edges(n + 1, src, dst, w, symmetric=True)
    net = rnmod.RoadNetwork.from_graph(g)
    net.set_tuning(hash_log2=11)
    net.set_profiling(times=True, work=False)
    R = np.array([0, 7, 150], dtype=np.int32)
    S = np.setdiff1d(np.arange(n + 1, dtype=np.int32), R)
    want = orc.dist_join(g, R, S, 200).pairs
    assert len(want) > 600
    assert_same(gpu_join(rnmod, net, R, S, 200), want)
    assert net.stats()["retried"] >= 1


def _colliding_ids(hb, V, count):
    """Vertex ids below V whose 24-bit Fibonacci hashes (the compact tables'
    bijection y -> y * 10368889 mod 2^24) share their top hb bits, so that all
    of them have the same home slot in a compact table of 2^hb slots."""
    inv = pow(10368889, -1, 1 << 24)
    shift = 24 - hb
    for home in range(1 << hb):
        z = np.arange(home << shift, (home + 1) << shift, dtype=np.int64)
        y = (z * inv) & 0xFFFFFF
        y = np.sort(y[y < V])
        if len(y) >= count:
            return y[:count]
    raise AssertionError("no home slot has enough ids below V")


@pytest.mark.parametrize("hb", [10, 11])
def test_probe_sequences_beyond_the_compact_field_go_to_the_next_tier(rnmod, orc, rg, hb):
    # a star whose 24 leaves all hash to one home slot of the first (compact)
    # table: a slot's probe-distance field counts at most 15 slots on, so the
    # search from the centre gives up on that tier and is re-run on the next;
    # the pairs are still exact
    V = 1 << 16
    leaves = _colliding_ids(hb, V, 24)
    centre = int(np.setdiff1d(np.arange(V), leaves)[0])
    rng = np.random.default_rng(31)
    w = rng.integers(3, 50, size=len(leaves))
    g = rg.from_edges(V, np.full(len(leaves), centre), leaves, w, symmetric=True)
    net = rnmod.RoadNetwork.from_graph(g)
    net.set_tuning(hash_log2=hb)
    net.set_profiling(times=True, work=False)
    R = np.array([centre, leaves[0]], dtype=np.int32)
    S = np.setdiff1d(np.concatenate([[centre], leaves]).astype(np.int32), R)
    want = orc.dist_join(g, R, S, 120).pairs
    assert len(want) > 30
    assert_same(gpu_join(rnmod, net, R, S, 120), want)
    assert net.stats()["retried"] >= 1


def test_global_tier_for_searches_beyond_lds(rnmod, orc, rg):
    g = rg.road_graph(128, 0)                    # ~16k vertices: a whole-graph ball
    net = rnmod.RoadNetwork.from_graph(g)        # outgrows every on-chip table
    R, S = rg.sample_disjoint(g.V, 40, 4000, 16)
    net.set_profiling(times=True, work=True)
    ref = orc.dist_join(g, R, S, 0xFFFFFFFE)
    assert_same(gpu_join(rnmod, net, R, S, 0xFFFFFFFE), ref.pairs)
    st = net.stats()
    assert st["global_searches"] == 40
    assert st["settled"] == ref.settled and st["arcs"] == ref.arcs


def test_directed_multigraph_with_zero_weights(rnmod, orc, rg):
    g = rg.random_digraph(3000, 12000, 4, wmin=1, wmax=60, zero_frac=0.2)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 200, 700, 5)
    for theta in (0, 10, 40, 90):
        assert_same(gpu_join(rnmod, net, R, S, theta), orc.dist_join(g, R, S, theta).pairs)


def test_disconnected_graph(rnmod, orc, rg):
    g = rg.road_graph(80, 3, p_drop=0.45, keep_lcc=False)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 500, 500, 6)
    assert_same(gpu_join(rnmod, net, R, S, 5000), orc.dist_join(g, R, S, 5000).pairs)


def test_one_distance_bin_beyond_2_16_records(rnmod, orc, rg):
    # 300 sources with an arc of weight 5 to each of 300 targets: 90 000 pairs
    # in the one (query, dist = 5) bin of the bucket sort (the chain adds 19
    # distinct weights, so the graph counts as varied and the bucket sort
    # runs); places in a bin past 2^16 - 1 are assigned by the bin's cursor
    R = np.arange(300, dtype=np.int32)
    S = np.arange(300, 600, dtype=np.int32)
    chain = np.arange(600, 619)
    g = rg.from_edges(620, np.concatenate([np.repeat(R, 300), chain]),
                      np.concatenate([np.tile(S, 300), chain + 1]),
                      np.concatenate([np.full(90000, 5), np.arange(1, 20)]), symmetric=False)
    net = rnmod.RoadNetwork.from_graph(g)
    for theta in (5, 12):
        want = orc.dist_join(g, R, S, theta).pairs
        assert want.shape[0] == 90000
        assert_same(gpu_join(rnmod, net, R, S, theta), want)


def test_oversized_bins_take_the_radix_sort_everywhere(rnmod, orc, rg):
    # bins past the bucket ranking's bound (4096 records) send the call's
    # scattered records to the radix sort: in a batch beside queries whose
    # bins are small, in a captured plan, in the request server and in the
    # allocation-free call, every result equals the oracle's; so do
    # k-closest-pairs calls with more tied candidates than the small sort holds
    import ctypes as C
    import torch
    R = np.arange(300, dtype=np.int32)
    S = np.arange(300, 600, dtype=np.int32)
    chain = np.arange(600, 619)
    g = rg.from_edges(620, np.concatenate([np.repeat(R, 300), chain]),
                      np.concatenate([np.tile(S, 300), chain + 1]),
                      np.concatenate([np.full(90000, 5), np.arange(1, 20)]), symmetric=False)
    net = rnmod.RoadNetwork.from_graph(g)
    specs = [{"R": R, "S": S, "theta": 12}, {"R": R[:50], "S": S[:60], "theta": 5},
             {"R": chain[:5].astype(np.int32), "S": chain[5:].astype(np.int32) + 1, "theta": 100},
             {"R": R[:70], "S": S[:40], "theta": 4}]
    wants = [orc.dist_join(g, sp["R"], sp["S"], sp["theta"]).pairs for sp in specs]
    assert [len(w) for w in wants][:2] == [90000, 3000]

    def check_batch(pairs, off):
        got = rnmod.pairs_to_numpy(pairs)
        for i, w in enumerate(wants):
            assert_same(got[off[i]:off[i + 1]], w)
    check_batch(*net.join_batch(specs)[:2])
    q, keep = net.make_queries(specs)
    plan = net.plan(q)
    for _ in range(2):
        check_batch(*plan.run()[:2])
    plan.close()
    srv = rnmod.Server(net, lanes=2, max_batch=4)
    ids = [srv.submit(sp["R"], sp["S"], sp["theta"], 0) for sp in specs]
    for i, w in zip(ids, wants):
        got, _ = srv.wait(i, guess=len(w) + 1)
        assert_same(got, w)
    srv.close()
    lib = rnmod.load_library()
    Rd, Sd = torch.as_tensor(R, device="cuda"), torch.as_tensor(S, device="cuda")
    out = torch.zeros((90001, 3), dtype=torch.int32, device="cuda")
    n = C.c_int64()
    st = lib.rn_dist_join_noalloc(net._h, C.c_void_p(Rd.data_ptr()), 300, C.c_void_p(Sd.data_ptr()), 300,
                                  C.c_uint32(12), C.c_void_p(out.data_ptr()), 90001, C.byref(n),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == rnmod.RN_OK and n.value == 90000
    assert_same(rnmod.pairs_to_numpy(out[:90000]), wants[0])
    # k-closest pairs whose ties at the bound give more candidates than the
    # one-block sort holds (90 000 pairs at distance 5): the radix sort runs
    for k in (10, 2048):
        assert_same(rnmod.pairs_to_numpy(net.kcp_join(R, S, k)), orc.kcp_join(g, R, S, k))


def test_lattice_closed_form_at_scale(rnmod, rg):
    side, c = 1024, 100
    g = rg.full_lattice(side, c)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 4096, 4096, 12)
    theta = 2000
    ri, rj = np.divmod(R.astype(np.int64), side)
    si, sj = np.divmod(S.astype(np.int64), side)
    rows = []
    for a in range(0, len(R), 512):
        d = c * (np.abs(ri[a:a + 512, None] - si[None, :]) + np.abs(rj[a:a + 512, None] - sj[None, :]))
        ia, ib = np.nonzero(d <= theta)
        rows.append(np.stack([d[ia, ib], R[a + ia], S[ib]], axis=1))
    want = np.concatenate(rows)
    want = want[np.lexsort((want[:, 2], want[:, 1], want[:, 0]))]
    got = gpu_join(rnmod, net, R, S, theta)
    assert got.shape[0] == want.shape[0]
    assert np.array_equal(got["dist"], want[:, 0]) and np.array_equal(got["u"], want[:, 1])
    assert np.array_equal(got["v"], want[:, 2])


def test_single_source_single_target_and_empty(rnmod, orc, rg, g64):
    net = rnmod.RoadNetwork.from_graph(g64)
    R, S = rg.sample_disjoint(g64.V, 1, 1, 13)
    d = int(orc.sssp(g64, int(R[0]))[S[0]])
    assert_same(gpu_join(rnmod, net, R, S, d), orc.dist_join(g64, R, S, d).pairs)
    assert gpu_join(rnmod, net, R, S, d).shape[0] == 1
    assert gpu_join(rnmod, net, R, S, d - 1).shape[0] == 0


def test_capacity_two_call_convention(rnmod, orc, rg, g64, torch_cuda):
    import ctypes as C
    torch = torch_cuda
    net = rnmod.RoadNetwork.from_graph(g64)
    R, S = rg.sample_disjoint(g64.V, 64, 64, 1)
    want = orc.dist_join(g64, R, S, 1500).pairs
    lib = rnmod.load_library()
    Rd = torch.as_tensor(R, device="cuda")
    Sd = torch.as_tensor(S, device="cuda")
    small = torch.zeros((5, 3), dtype=torch.int32, device="cuda")
    n = C.c_int64()
    st = lib.rn_dist_join(net._h, C.c_void_p(Rd.data_ptr()), 64, C.c_void_p(Sd.data_ptr()), 64, 1500,
                          C.c_void_p(small.data_ptr()), 5, C.byref(n), None)
    assert st == rnmod.RN_ERR_CAPACITY and n.value == len(want)
    assert torch.count_nonzero(small).item() == 0        # nothing written on failure
    big = torch.zeros((len(want), 3), dtype=torch.int32, device="cuda")
    st = lib.rn_dist_join(net._h, C.c_void_p(Rd.data_ptr()), 64, C.c_void_p(Sd.data_ptr()), 64, 1500,
                          C.c_void_p(big.data_ptr()), len(want), C.byref(n), None)
    assert st == rnmod.RN_OK
    assert_same(rnmod.pairs_to_numpy(big), want)


@pytest.mark.parametrize("case", ["dup_R", "dup_S", "overlap", "range_R", "range_S", "negative"])
def test_argument_errors_then_recovery(rnmod, orc, rg, g64, case):
    net = rnmod.RoadNetwork.from_graph(g64)
    R, S = rg.sample_disjoint(g64.V, 64, 64, 1)
    R, S = R.copy(), S.copy()
    if case == "dup_R":
        R[5] = R[9]
    elif case == "dup_S":
        S[1] = S[0]
    elif case == "overlap":
        R[3] = S[7]
    elif case == "range_R":
        R[0] = g64.V
    elif case == "range_S":
        S[63] = g64.V + 100
    else:
        R[2] = -1
    with pytest.raises(rnmod.RnError) as ei:
        net.dist_join(R, S, 1500)
    assert ei.value.status == rnmod.RN_ERR_ARG
    R2, S2 = rg.sample_disjoint(g64.V, 64, 64, 1)
    assert_same(gpu_join(rnmod, net, R2, S2, 1500), orc.dist_join(g64, R2, S2, 1500).pairs)


def test_partition_order_never_changes_results(rnmod, orc, rg):
    g = rg.road_graph(160, 1)
    R, S = rg.sample_disjoint(g.V, 2000, 2000, 14)
    want = orc.dist_join(g, R, S, 2500).pairs
    net = rnmod.RoadNetwork.from_graph(g)
    assert_same(gpu_join(rnmod, net, R, S, 2500), want)
    for alpha, leaf in ((1.0, 256), (0.5, 64), (1.0, 1)):
        part = net.partition(alpha, leaf)
        assert part.shape == (g.V,)
        assert_same(gpu_join(rnmod, net, R, S, 2500), want)


def test_repeatable_and_stream_argument(rnmod, orc, rg, g64, torch_cuda):
    torch = torch_cuda
    net = rnmod.RoadNetwork.from_graph(g64)
    R, S = rg.sample_disjoint(g64.V, 200, 200, 15)
    want = orc.dist_join(g64, R, S, 2000).pairs
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = rnmod.pairs_to_numpy(net.dist_join(R, S, 2000, stream=s))
    b = gpu_join(rnmod, net, R, S, 2000)
    assert_same(a, want)
    assert_same(b, want)


def test_profiling_stats(rnmod, rg, g64):
    net = rnmod.RoadNetwork.from_graph(g64)
    net.set_profiling(True)
    R, S = rg.sample_disjoint(g64.V, 64, 64, 1)
    out = net.dist_join(R, S, 1500)
    st = net.stats()
    assert st["pairs"] == out.shape[0]
    assert st["relax_ms"] > 0 and st["total_ms"] >= st["relax_ms"]


@pytest.mark.parametrize("graph", ["road", "directed"])
def test_searches_from_the_smaller_side(rnmod, orc, rg, graph):
    # |S| < |R|: the library searches from S over the reversed arcs; a directed
    # graph with zero weights makes the reversal visible if it were wrong
    if graph == "road":
        g = rg.road_graph(96, 4)
    else:
        g = rg.random_digraph(3000, 12000, 31, wmin=1, wmax=60, zero_frac=0.2)
    net = rnmod.RoadNetwork.from_graph(g)
    R, S = rg.sample_disjoint(g.V, 900, 60, 32)
    for theta in (0, 40, 1500, 0xFFFFFFFE):
        want = orc.dist_join(g, R, S, theta).pairs
        assert_same(gpu_join(rnmod, net, R, S, theta), want)
        out, off, status = net.join_batch([{"R": R, "S": S, "theta": theta, "forward": True},
                                           {"R": R, "S": S, "theta": theta}])
        segs = rnmod.split_batch(out, off)
        assert_same(segs[0], want)
        assert_same(segs[1], want)
    for k in (1, 77, 5000):
        assert_same(rnmod.pairs_to_numpy(net.kcp_join(R, S, k)), orc.kcp_join(g, R, S, k))
    # argument errors name the caller's sets
    S2 = S.copy()
    S2[1] = S2[0]
    with pytest.raises(rnmod.RnError) as ei:
        net.dist_join(R, S2, 100)
    assert "duplicate in S" in str(ei.value)


def shuffled(rg, g, seed):
    """The same graph with its vertex ids permuted (no locality left in them)."""
    return rg.shuffle_ids(g, seed)[0]


@pytest.mark.parametrize("graph", ["road", "directed"])
def test_renumbered_device_copy(rnmod, orc, rg, graph):
    # rn_partition renumbers the device copy in leaf order when that is more
    # local than the loaded ids (shuffled ids here); R, S and the pairs stay in
    # the caller's ids, also for searches from S over the reversed arcs
    # (directed graph), through the global tier (theta = max) and for k closest
    # pairs answered by direct arcs or by searches
    if graph == "road":
        g = shuffled(rg, rg.road_graph(96, 4), 40)
    else:
        g = rg.random_digraph(3000, 12000, 33, wmin=1, wmax=60, zero_frac=0.2)
    net = rnmod.RoadNetwork.from_graph(g)
    assert not net.renumbered(0)
    net.partition(0.5, 64)
    assert net.renumbered(0)
    for nR, nS, seed in ((900, 60, 34), (60, 900, 35)):
        R, S = rg.sample_disjoint(g.V, nR, nS, seed)
        for theta in (0, 40, 1500, 0xFFFFFFFE):
            assert_same(gpu_join(rnmod, net, R, S, theta), orc.dist_join(g, R, S, theta).pairs)
        for k in (1, 77, 5000):
            assert_same(rnmod.pairs_to_numpy(net.kcp_join(R, S, k)), orc.kcp_join(g, R, S, k))
    # a second partition renumbers again, from the caller's numbering
    net.partition(1.0, 256)
    assert net.renumbered(0)
    R, S = rg.sample_disjoint(g.V, 500, 500, 36)
    assert_same(gpu_join(rnmod, net, R, S, 2000), orc.dist_join(g, R, S, 2000).pairs)


def test_local_numbering_is_kept(rnmod, orc, rg):
    # a road graph numbered row by row is already more local than leaf order
    g = rg.road_graph(96, 4)
    net = rnmod.RoadNetwork.from_graph(g)
    net.partition(1.0, 64)
    assert not net.renumbered(0)
    R, S = rg.sample_disjoint(g.V, 400, 400, 39)
    assert_same(gpu_join(rnmod, net, R, S, 2000), orc.dist_join(g, R, S, 2000).pairs)


def test_renumbered_handle_of_several_graphs_and_plans(rnmod, orc, rg):
    # per-graph id ranges of a multi-graph handle; a plan captured before the
    # partition keeps answering correctly after it (the device copy is
    # renumbered in place)
    g1, g2 = rg.road_graph(64, 5), shuffled(rg, rg.road_graph(80, 6), 41)   # only g2 is renumbered
    net = rnmod.RoadNetwork.from_graphs([g1, g2])
    R1, S1 = rg.sample_disjoint(g1.V, 300, 200, 37)
    R2, S2 = rg.sample_disjoint(g2.V, 200, 300, 38)
    specs = [{"R": R1, "S": S1, "theta": 1800, "graph": 0}, {"R": R2, "S": S2, "theta": 2200, "graph": 1},
             {"R": R2, "S": S2, "k": 40, "graph": 1}]
    wants = [orc.dist_join(g1, R1, S1, 1800).pairs, orc.dist_join(g2, R2, S2, 2200).pairs,
             orc.kcp_join(g2, R2, S2, 40)]
    q, keep = net.make_queries(specs)
    plan = net.plan(q)
    for part in (None, (0.25, 32), (1.0, 128)):
        if part:
            net.partition(*part)
            assert not net.renumbered(0) and net.renumbered(1)
        out, off, status = net.join_batch(q)
        assert not status.any()
        for got, want in zip(rnmod.split_batch(out, off), wants):
            assert_same(got, want)
        out, off, status = plan.run()
        assert not status.any()
        for got, want in zip(rnmod.split_batch(out, off), wants):
            assert_same(got, want)
    plan.close()
