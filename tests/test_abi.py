"""The C-ABI library loads and exports every symbol include/rn.h declares.

No device work here: only calls that fail argument checks before touching a
GPU, plus the host-only partitioner entry point.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rn.h")


@pytest.fixture(scope="module")
def rn():
    from paper_1607_07696_amd import rn
    rn.load_library()
    return rn


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rn_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree(rn):
    decl = declared_functions()
    assert decl == sorted(rn.EXPORTS)


def test_every_declared_symbol_is_exported(rn):
    lib = rn.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_pair_layout_matches_header(rn):
    assert rn.PAIR_DTYPE.itemsize == 12


def test_graph_load_rejects_malformed_csr_before_device(rn):
    lib = rn.load_library()
    h = C.c_void_p()
    rp = np.array([0, 1, 3], dtype=np.int32)
    col = np.array([1, 0, 5], dtype=np.int32)   # 5 is out of range
    w = np.array([1, 1, 1], dtype=np.uint32)
    i32 = C.POINTER(C.c_int32)
    st = lib.rn_graph_load(2, 3, rp.ctypes.data_as(i32), col.ctypes.data_as(i32),
                           w.ctypes.data_as(C.POINTER(C.c_uint32)), C.byref(h))
    assert st == rn.RN_ERR_ARG and not h.value
    assert b"col" in lib.rn_last_error()
    rp_bad = np.array([0, 2, 1], dtype=np.int32)
    st = lib.rn_graph_load(2, 1, rp_bad.ctypes.data_as(i32), col.ctypes.data_as(i32),
                           w.ctypes.data_as(C.POINTER(C.c_uint32)), C.byref(h))
    assert st == rn.RN_ERR_ARG
    st = lib.rn_graph_load(0, 0, rp.ctypes.data_as(i32), None, None, C.byref(h))
    assert st == rn.RN_ERR_ARG


def test_join_calls_reject_null_handle(rn):
    lib = rn.load_library()
    n = C.c_int64(7)
    st = lib.rn_dist_join(None, None, 1, None, 1, 5, None, 0, C.byref(n), None)
    assert st == rn.RN_ERR_ARG and n.value == 0
    st = lib.rn_kcp_join(None, None, 1, None, 1, 5, None, 0, C.byref(n), None)
    assert st == rn.RN_ERR_ARG
    assert lib.rn_set_tuning(None, 0, 11) == rn.RN_ERR_ARG
    assert lib.rn_graph_num_vertices(None) == 0
    lib.rn_graph_free(None)


def test_partition_host_argument_checks(rn, rg):
    g = rg.road_graph(8, 0)
    with pytest.raises(rn.RnError):
        rn.partition_host(g.row_ptr, g.col, g.w, alpha=1.5)
    with pytest.raises(rn.RnError):
        rn.partition_host(g.row_ptr, g.col, g.w, max_leaf=0)


def test_version(rn):
    assert rn.load_library().rn_version().startswith(b"rn ")


def test_batch_calls_reject_bad_arguments_before_device(rn):
    lib = rn.load_library()
    off = np.ones(3, dtype=np.int64)
    i64 = C.POINTER(C.c_int64)
    q = (rn.Query * 2)()
    st = lib.rn_join_batch(None, q, 2, None, 0, off.ctypes.data_as(i64), None, None)
    assert st == rn.RN_ERR_ARG
    assert lib.rn_join_batch(None, q, 2, None, 0, None, None, None) == rn.RN_ERR_ARG
    assert lib.rn_autotune(None, q, 2, 64, None) == rn.RN_ERR_ARG
    h = C.c_void_p(1)
    assert lib.rn_plan_create(None, q, 2, None, 0, None, C.byref(h)) == rn.RN_ERR_ARG and not h.value
    assert lib.rn_plan_run(None, off.ctypes.data_as(i64), None, None) == rn.RN_ERR_ARG
    lib.rn_plan_free(None)
    assert lib.rn_graph_count(None) == 0
    assert lib.rn_graph_size(None, 0, None, None) == rn.RN_ERR_ARG


def test_graph_load_many_names_the_bad_graph(rn, rg):
    lib = rn.load_library()
    good = rg.road_graph(8, 0)
    bad_col = good.col.copy()
    bad_col[0] = good.V + 3
    graphs = [(good.row_ptr, good.col, good.w), (good.row_ptr, bad_col, good.w)]
    V = np.array([good.V, good.V], dtype=np.int32)
    A = np.array([good.A, good.A], dtype=np.int64)
    ptrs = [(C.c_void_p * 2)(*[np.ascontiguousarray(x[j]).ctypes.data for x in graphs]) for j in range(3)]
    h = C.c_void_p()
    st = lib.rn_graph_load_many(2, V.ctypes.data_as(C.POINTER(C.c_int32)), A.ctypes.data_as(C.POINTER(C.c_int64)),
                                *ptrs, C.byref(h))
    assert st == rn.RN_ERR_ARG and not h.value
    assert lib.rn_last_error().startswith(b"graph 1:")


def test_query_struct_layout(rn):
    assert C.sizeof(rn.Query) == 48
    assert rn.Query.nR.offset == 16 and rn.Query.hash_log2.offset == 40


def test_server_calls_reject_bad_arguments_before_device(rn):
    lib = rn.load_library()
    h = C.c_void_p(1)
    cfg = rn.ServerConfig(0, 2, 8, 4, 1 << 30)
    assert lib.rn_server_create(None, C.byref(cfg), C.byref(h)) == rn.RN_ERR_ARG and not h.value
    rid = C.c_int64(5)
    R = np.array([1, 2], dtype=np.int32)
    i32 = C.POINTER(C.c_int32)
    assert lib.rn_server_submit(None, R.ctypes.data_as(i32), 2, R.ctypes.data_as(i32), 2, 10, 0,
                                C.byref(rid)) == rn.RN_ERR_ARG
    assert rid.value == 0
    n = C.c_int64(3)
    assert lib.rn_server_wait(None, 1, None, 0, C.byref(n), None) == rn.RN_ERR_ARG and n.value == 0
    assert lib.rn_server_get_stats(None, None) == rn.RN_ERR_ARG
    lib.rn_server_free(None)
    assert C.sizeof(rn.ServerConfig) == 32 and C.sizeof(rn.ServerStats) == 64


def test_header_constants_match_binding(rn):
    text = open(HEADER).read()
    for name in ("RN_TABLE_GLOBAL", "RN_QUERY_FORWARD"):
        m = re.search(r"#define\s+" + name + r"\s+(\w+)", text)
        assert m and int(m.group(1), 0) == getattr(rn, name), name
