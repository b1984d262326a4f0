"""Thin ctypes binding of librn (include/rn.h).

Argument marshalling only: every step of a join runs in the library's HIP
kernels.  torch supplies device memory and the current stream.  If librn.so
has not been built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librn.so")

RN_OK, RN_ERR_ARG, RN_ERR_NOMEM, RN_ERR_CAPACITY, RN_ERR_DEVICE, RN_ERR_BUSY = 0, -1, -2, -3, -4, -5
RN_PROFILE_TIMES, RN_PROFILE_WORK = 1, 2
PAIR_DTYPE = np.dtype([("u", "<i4"), ("v", "<i4"), ("dist", "<u4")])

# Every symbol include/rn.h declares.
EXPORTS = (
    "rn_graph_load", "rn_graph_free", "rn_graph_num_vertices", "rn_graph_num_arcs",
    "rn_partition_host", "rn_partition", "rn_dist_join", "rn_kcp_join",
    "rn_set_tuning", "rn_get_tuning", "rn_set_profiling", "rn_last_stats",
    "rn_last_error", "rn_version",
)


class RnError(RuntimeError):
    def __init__(self, status: int, msg: str, needed: int | None = None):
        super().__init__(f"rn status {status}: {msg}")
        self.status, self.needed = status, needed


class Stats(C.Structure):
    _fields_ = [("stage_ms", C.c_float), ("relax_ms", C.c_float), ("retry_ms", C.c_float),
                ("select_ms", C.c_float), ("sort_ms", C.c_float), ("total_ms", C.c_float),
                ("pairs", C.c_int64), ("arcs", C.c_int64), ("settled", C.c_int64),
                ("retried", C.c_int32), ("global_searches", C.c_int32),
                ("relax_launches", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librn.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first")
    lib = C.CDLL(path)
    i32p, u32p, i64p, vp = C.POINTER(C.c_int32), C.POINTER(C.c_uint32), C.POINTER(C.c_int64), C.c_void_p
    lib.rn_graph_load.argtypes = [C.c_int32, C.c_int64, i32p, i32p, u32p, C.POINTER(vp)]
    lib.rn_graph_free.argtypes = [vp]
    lib.rn_graph_free.restype = None
    lib.rn_graph_num_vertices.argtypes = [vp]
    lib.rn_graph_num_arcs.argtypes = [vp]
    lib.rn_graph_num_arcs.restype = C.c_int64
    lib.rn_partition_host.argtypes = [C.c_int32, C.c_int64, i32p, i32p, u32p, C.c_float, C.c_int32,
                                      i32p, i32p]
    lib.rn_partition.argtypes = [vp, C.c_float, C.c_int32, i32p]
    lib.rn_dist_join.argtypes = [vp, vp, C.c_int32, vp, C.c_int32, C.c_uint32, vp, C.c_int64, i64p, vp]
    lib.rn_kcp_join.argtypes = [vp, vp, C.c_int32, vp, C.c_int32, C.c_int32, vp, C.c_int64, i64p, vp]
    lib.rn_set_tuning.argtypes = [vp, C.c_int64, C.c_int32]
    lib.rn_get_tuning.argtypes = [vp, u32p, i32p]
    lib.rn_set_profiling.argtypes = [vp, C.c_int32]
    lib.rn_last_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.rn_last_error.restype = C.c_char_p
    lib.rn_version.restype = C.c_char_p
    for name in ("rn_graph_load", "rn_graph_num_vertices", "rn_partition_host", "rn_partition",
                 "rn_dist_join", "rn_kcp_join", "rn_set_tuning", "rn_get_tuning",
                 "rn_set_profiling", "rn_last_stats"):
        getattr(lib, name).restype = C.c_int32
    _lib = lib
    return lib


def _check(status: int, needed: int | None = None):
    if status != RN_OK:
        raise RnError(status, load_library().rn_last_error().decode(), needed)


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    ptype = {np.int32: C.c_int32, np.uint32: C.c_uint32}[np.dtype(dtype).type]
    return a, a.ctypes.data_as(C.POINTER(ptype))


def partition_host(row_ptr, col, w, alpha: float = 0.0, max_leaf: int = 256):
    """Host recursive bisection; returns (part, order) as int32 arrays."""
    lib = load_library()
    rp, rpp = _host(row_ptr, np.int32)
    cl, clp = _host(col, np.int32)
    ww, wp = _host(w, np.uint32)
    V = rp.shape[0] - 1
    part = np.empty(V, dtype=np.int32)
    order = np.empty(V, dtype=np.int32)
    _check(lib.rn_partition_host(V, cl.shape[0], rpp, clp, wp, float(alpha), int(max_leaf),
                                 part.ctypes.data_as(C.POINTER(C.c_int32)),
                                 order.ctypes.data_as(C.POINTER(C.c_int32))))
    return part, order


def pairs_to_numpy(t) -> np.ndarray:
    """Device pair tensor [n, 3] (int32 u, v, dist bits) -> structured numpy array."""
    a = t.detach().to("cpu").contiguous().numpy()
    return a.view(PAIR_DTYPE).reshape(-1) if a.size else np.zeros(0, dtype=PAIR_DTYPE)


class RoadNetwork:
    """A graph resident on the current HIP device (an rn_graph handle)."""

    def __init__(self, row_ptr, col, w):
        lib = load_library()
        rp, rpp = _host(row_ptr, np.int32)
        cl, clp = _host(col, np.int32)
        ww, wp = _host(w, np.uint32)
        h = C.c_void_p()
        _check(lib.rn_graph_load(rp.shape[0] - 1, cl.shape[0], rpp, clp, wp, C.byref(h)))
        self._h = h
        self.V = rp.shape[0] - 1
        self.A = cl.shape[0]
        self._out = None

    @classmethod
    def from_graph(cls, g) -> "RoadNetwork":
        return cls(g.row_ptr, g.col, g.w)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().rn_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- knobs
    def partition(self, alpha: float = 0.0, max_leaf: int = 256) -> np.ndarray:
        part = np.empty(self.V, dtype=np.int32)
        _check(load_library().rn_partition(self._h, float(alpha), int(max_leaf),
                                           part.ctypes.data_as(C.POINTER(C.c_int32))))
        return part

    def set_tuning(self, delta: int = -1, hash_log2: int = -1):
        _check(load_library().rn_set_tuning(self._h, int(delta), int(hash_log2)))

    def tuning(self) -> tuple[int, int]:
        d, h = C.c_uint32(), C.c_int32()
        _check(load_library().rn_get_tuning(self._h, C.byref(d), C.byref(h)))
        return d.value, h.value

    def set_profiling(self, times: bool = True, work: bool = False):
        flags = (RN_PROFILE_TIMES if times else 0) | (RN_PROFILE_WORK if work else 0)
        _check(load_library().rn_set_profiling(self._h, flags))

    def stats(self) -> dict:
        s = Stats()
        _check(load_library().rn_last_stats(self._h, C.byref(s)))
        return s.as_dict()

    # -------------------------------------------------------------- joins
    @staticmethod
    def _dev_ids(x):
        import torch
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32))
        if x.dtype != torch.int32:
            x = x.to(torch.int32)
        if not x.is_cuda:
            x = x.to("cuda")
        return x.contiguous()

    def _out_buffer(self, n: int):
        import torch
        if self._out is None or self._out.shape[0] < n:
            self._out = torch.empty((max(n, 1024), 3), dtype=torch.int32, device="cuda")
        return self._out

    def _call(self, fn, R, S, arg, stream):
        import torch
        R, S = self._dev_ids(R), self._dev_ids(S)
        if stream is None:
            stream = torch.cuda.current_stream()
        sptr = C.c_void_p(stream.cuda_stream)
        n = C.c_int64()
        out = self._out_buffer(0)
        st = fn(self._h, C.c_void_p(R.data_ptr()), R.numel(), C.c_void_p(S.data_ptr()), S.numel(),
                arg, C.c_void_p(out.data_ptr()), out.shape[0], C.byref(n), sptr)
        if st == RN_ERR_CAPACITY and n.value > out.shape[0]:
            out = self._out_buffer(n.value)
            st = fn(self._h, C.c_void_p(R.data_ptr()), R.numel(), C.c_void_p(S.data_ptr()), S.numel(),
                    arg, C.c_void_p(out.data_ptr()), out.shape[0], C.byref(n), sptr)
        _check(st, n.value)
        return out[: n.value]

    def dist_join(self, R, S, theta: int, stream=None):
        """Theta-join on the device: int32 tensor [n, 3] of (u, v, dist) sorted by (dist, u, v).

        The returned view aliases an internal buffer reused by the next call."""
        return self._call(load_library().rn_dist_join, R, S, C.c_uint32(int(theta)), stream)

    def kcp_join(self, R, S, k: int, stream=None):
        """k closest pairs on the device: int32 tensor [n, 3], n = min(k, reachable pairs)."""
        return self._call(load_library().rn_kcp_join, R, S, C.c_int32(int(k)), stream)
