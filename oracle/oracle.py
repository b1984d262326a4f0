"""ctypes binding of the plain C oracle (``rn_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its Python binding.

``build()`` compiles ``rn_oracle.c`` with gcc into ``liborc.so`` next to this
file; the other functions load that library (building it if it is missing).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rn_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
UNREACH = 0xFFFFFFFF

PAIR_DTYPE = np.dtype([("u", "<i4"), ("v", "<i4"), ("dist", "<u4")])

_lib = None


def build(src: str = SRC, lib: str = LIB) -> str:
    """Compile the oracle source ``src`` into ``lib``; returns the library path."""
    tmp = lib + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-pthread", src, "-o", tmp])
    os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    _lib = open_library(LIB)
    return _lib


def open_library(path: str):
    """Load an oracle build (the default one, or a variant compiled by a test)."""
    lib = C.CDLL(path)
    i32p, u32p = C.POINTER(C.c_int32), C.POINTER(C.c_uint32)
    i64p = C.POINTER(C.c_int64)
    pp = C.POINTER(C.c_void_p)
    lib.orc_dist_join.argtypes = [C.c_int32, i32p, i32p, u32p, i32p, C.c_int32, i32p, C.c_int32,
                                  C.c_uint32, C.c_int, pp, i64p, i64p, i64p]
    lib.orc_dist_join.restype = C.c_int
    lib.orc_kcp_join.argtypes = [C.c_int32, i32p, i32p, u32p, i32p, C.c_int32, i32p, C.c_int32,
                                 C.c_int32, pp, i64p]
    lib.orc_kcp_join.restype = C.c_int
    lib.orc_sssp.argtypes = [C.c_int32, i32p, i32p, u32p, C.c_int32, C.c_uint32, u32p]
    lib.orc_sssp.restype = C.c_int
    lib.orc_object_join.argtypes = [C.c_int32, i32p, i32p, u32p, i32p, u32p, C.c_int32, i32p, u32p, C.c_int32,
                                    C.c_uint32, pp, i64p]
    lib.orc_object_join.restype = C.c_int
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_num_cores.restype = C.c_int
    return lib


def _arr(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    ptype = C.POINTER(C.c_int32) if dtype == np.int32 else C.POINTER(C.c_uint32)
    return a, a.ctypes.data_as(ptype)


def _graph_args(g):
    rp, rpp = _arr(g.row_ptr, np.int32)
    col, colp = _arr(g.col, np.int32)
    w, wp = _arr(g.w, np.uint32)
    return (rp, col, w), (C.c_int32(g.V), rpp, colp, wp)


def _take_pairs(lib, ptr: C.c_void_p, n: int) -> np.ndarray:
    if n == 0 or not ptr.value:
        if ptr.value:
            lib.orc_free(ptr)
        return np.zeros(0, dtype=PAIR_DTYPE)
    buf = (C.c_char * (n * PAIR_DTYPE.itemsize)).from_address(ptr.value)
    out = np.frombuffer(buf, dtype=PAIR_DTYPE).copy()
    lib.orc_free(ptr)
    return out


def num_cores() -> int:
    return int(_load().orc_num_cores())


class JoinResult:
    """Sorted pairs plus the work counts of the searches that produced them."""

    def __init__(self, pairs, arcs, settled, seconds, threads):
        self.pairs, self.arcs, self.settled = pairs, arcs, settled
        self.seconds, self.threads = seconds, threads


def dist_join(g, R, S, theta: int, threads: int = 0, lib=None) -> JoinResult:
    """Theta-join: every (u, v, dist) with u in R, v in S, dist <= theta, sorted by (dist,u,v)."""
    lib = lib or _load()
    keep, gargs = _graph_args(g)
    R, Rp = _arr(R, np.int32)
    S, Sp = _arr(S, np.int32)
    out, n, arcs, settled = C.c_void_p(), C.c_int64(), C.c_int64(), C.c_int64()
    nthr = threads if threads > 0 else int(lib.orc_num_cores())
    t0 = time.perf_counter()
    rc = lib.orc_dist_join(*gargs, Rp, len(R), Sp, len(S), C.c_uint32(int(theta)), nthr,
                           C.byref(out), C.byref(n), C.byref(arcs), C.byref(settled))
    dt = time.perf_counter() - t0
    if rc != 0:
        raise ValueError("oracle theta-join rejected its arguments")
    del keep
    return JoinResult(_take_pairs(lib, out, n.value), arcs.value, settled.value, dt,
                      min(nthr, max(1, len(R))))


def kcp_join(g, R, S, k: int, lib=None) -> np.ndarray:
    """k closest pairs under (dist,u,v), sorted; fewer if fewer pairs are reachable."""
    lib = lib or _load()
    keep, gargs = _graph_args(g)
    R, Rp = _arr(R, np.int32)
    S, Sp = _arr(S, np.int32)
    out, n = C.c_void_p(), C.c_int64()
    rc = lib.orc_kcp_join(*gargs, Rp, len(R), Sp, len(S), int(k), C.byref(out), C.byref(n))
    if rc != 0:
        raise ValueError("oracle k-closest-pairs join rejected its arguments")
    del keep
    return _take_pairs(lib, out, n.value)


def object_join(g, R_arc, R_off, S_arc, S_off, theta: int, lib=None) -> np.ndarray:
    """Theta-join of objects on edges (object = arc index + distance from its
    tail; see ``rn_oracle.c``): (i, j, dist) for R object i and S object j with
    dist <= theta, sorted by (dist, i, j)."""
    lib = lib or _load()
    keep, gargs = _graph_args(g)
    Ra, Rap = _arr(R_arc, np.int32)
    Ro, Rop = _arr(R_off, np.uint32)
    Sa, Sap = _arr(S_arc, np.int32)
    So, Sop = _arr(S_off, np.uint32)
    out, n = C.c_void_p(), C.c_int64()
    rc = lib.orc_object_join(*gargs, Rap, Rop, len(Ra), Sap, Sop, len(Sa), C.c_uint32(int(theta)),
                             C.byref(out), C.byref(n))
    if rc != 0:
        raise ValueError("oracle object join rejected its arguments")
    del keep
    return _take_pairs(lib, out, n.value)


def sssp(g, src: int, cutoff: int = UNREACH - 1, lib=None) -> np.ndarray:
    """Distances from ``src`` (uint32; ``UNREACH`` beyond ``cutoff`` or unreachable)."""
    lib = lib or _load()
    keep, gargs = _graph_args(g)
    d = np.empty(g.V, dtype=np.uint32)
    rc = lib.orc_sssp(*gargs, int(src), C.c_uint32(int(cutoff)),
                      d.ctypes.data_as(C.POINTER(C.c_uint32)))
    if rc != 0:
        raise ValueError("oracle sssp rejected its arguments")
    del keep
    return d
