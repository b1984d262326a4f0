"""GPU test of rn_dist_join_noalloc, the theta-join whose device buffers all
come from one static device array: its output, through the C ABI, equals
rn_dist_join's (tolerance 0) on two calls in a row, the second smaller (on
another graph), and then again on the first graph."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1607_07696_amd import rn
    return torch, rn, rn.load_library()


def noalloc(torch, rn, lib, net, R, S, theta, cap):
    Rd = torch.as_tensor(np.asarray(R, dtype=np.int32), device="cuda")
    Sd = torch.as_tensor(np.asarray(S, dtype=np.int32), device="cuda")
    out = torch.zeros((max(cap, 1), 3), dtype=torch.int32, device="cuda")
    n = C.c_int64()
    st = lib.rn_dist_join_noalloc(net._h, C.c_void_p(Rd.data_ptr()), Rd.numel(), C.c_void_p(Sd.data_ptr()),
                                  Sd.numel(), C.c_uint32(theta), C.c_void_p(out.data_ptr()), cap, C.byref(n),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, n.value, out


def check(torch, rn, lib, net, R, S, theta):
    want = rn.pairs_to_numpy(net.dist_join(R, S, theta)).copy()
    st, n, out = noalloc(torch, rn, lib, net, R, S, theta, len(want) + 5)
    assert st == rn.RN_OK, lib.rn_last_error().decode()
    assert n == len(want)
    got = rn.pairs_to_numpy(out[:n])
    assert np.array_equal(got, want)
    return want


def test_noalloc_matches_dist_join(env, orc, rg):
    torch, rn, lib = env
    big = rg.road_graph(1024, 0)
    R, S = rg.sample_disjoint(big.V, 8192, 8192, 2)
    nb = rn.RoadNetwork.from_graph(big)
    print("noalloc: 1024x1024, 8192 x 8192, theta 3000", flush=True)
    a = check(torch, rn, lib, nb, R, S, 3000)
    assert len(a) == 76730
    small = rg.road_graph(64, 0)
    R2, S2 = rg.sample_disjoint(small.V, 64, 64, 1)
    ns = rn.RoadNetwork.from_graph(small)
    print("noalloc: 64x64, 64 x 64, theta 1500", flush=True)
    b = check(torch, rn, lib, ns, R2, S2, 1500)
    assert np.array_equal(b, orc.dist_join(small, R2, S2, 1500).pairs)
    print("noalloc: 1024x1024 again, 500 x 700, theta 2000", flush=True)
    check(torch, rn, lib, nb, R[:500], S[:700], 2000)
    # capacity and argument errors behave as rn_dist_join's
    st, n, _ = noalloc(torch, rn, lib, ns, R2, S2, 1500, 3)
    assert st == rn.RN_ERR_CAPACITY and n == len(b)
    Rbad = R2.copy()
    Rbad[0] = S2[0]
    st, _, _ = noalloc(torch, rn, lib, ns, Rbad, S2, 1500, 10)
    assert st == rn.RN_ERR_ARG
    check(torch, rn, lib, ns, R2, S2, 700)
