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
    "rn_partition_host", "rn_partition", "rn_graph_renumbered", "rn_dist_join", "rn_kcp_join",
    "rn_set_tuning", "rn_get_tuning", "rn_set_profiling", "rn_last_stats",
    "rn_last_error", "rn_version",
    "rn_graph_load_many", "rn_graph_count", "rn_graph_size", "rn_join_batch", "rn_autotune",
    "rn_plan_create", "rn_plan_run", "rn_plan_free",
    "rn_server_create", "rn_server_submit", "rn_server_wait", "rn_server_get_stats", "rn_server_free",
    "rn_objects_graph", "rn_dist_join_noalloc",
)
RN_DELTA_DEFAULT = 0xFFFFFFFF
RN_QUERY_FORWARD = 1
RN_TABLE_GLOBAL = 15
MAX_DIST = 0xFFFFFFFE


class RnError(RuntimeError):
    def __init__(self, status: int, msg: str, needed: int | None = None):
        super().__init__(f"rn status {status}: {msg}")
        self.status, self.needed = status, needed


class Query(C.Structure):
    """struct rn_query (include/rn.h)."""
    _fields_ = [("R", C.c_void_p), ("S", C.c_void_p), ("nR", C.c_int32), ("nS", C.c_int32),
                ("graph", C.c_int32), ("k", C.c_int32), ("theta", C.c_uint32), ("delta", C.c_uint32),
                ("hash_log2", C.c_int32), ("flags", C.c_int32)]


class ServerConfig(C.Structure):
    """struct rn_server_config (include/rn.h)."""
    _fields_ = [("graph", C.c_int32), ("lanes", C.c_int32), ("max_batch", C.c_int32),
                ("global_slots", C.c_int32), ("hbm_budget", C.c_int64), ("heavy_lane", C.c_int32),
                ("reserved", C.c_int32)]


class ServerStats(C.Structure):
    """struct rn_server_stats (include/rn.h)."""
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("reruns", C.c_int64), ("peak_budget", C.c_int64), ("device_bytes", C.c_int64),
                ("max_in_flight", C.c_int32), ("max_lanes_busy", C.c_int32), ("max_batch_seen", C.c_int32),
                ("budget_waits", C.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


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
    lib.rn_graph_renumbered.argtypes = [vp, C.c_int32]
    lib.rn_dist_join.argtypes = [vp, vp, C.c_int32, vp, C.c_int32, C.c_uint32, vp, C.c_int64, i64p, vp]
    lib.rn_kcp_join.argtypes = [vp, vp, C.c_int32, vp, C.c_int32, C.c_int32, vp, C.c_int64, i64p, vp]
    lib.rn_dist_join_noalloc.argtypes = [vp, vp, C.c_int32, vp, C.c_int32, C.c_uint32, vp, C.c_int64, i64p, vp]
    lib.rn_set_tuning.argtypes = [vp, C.c_int64, C.c_int32]
    lib.rn_get_tuning.argtypes = [vp, u32p, i32p]
    lib.rn_set_profiling.argtypes = [vp, C.c_int32]
    lib.rn_last_stats.argtypes = [vp, C.POINTER(Stats)]
    pp = C.POINTER(vp)
    lib.rn_graph_load_many.argtypes = [C.c_int32, i32p, i64p, pp, pp, pp, C.POINTER(vp)]
    lib.rn_graph_count.argtypes = [vp]
    lib.rn_graph_size.argtypes = [vp, C.c_int32, i32p, i64p]
    qp = C.POINTER(Query)
    lib.rn_join_batch.argtypes = [vp, qp, C.c_int32, vp, C.c_int64, i64p, i32p, vp]
    lib.rn_autotune.argtypes = [vp, qp, C.c_int32, C.c_int32, vp]
    lib.rn_plan_create.argtypes = [vp, qp, C.c_int32, vp, C.c_int64, vp, C.POINTER(vp)]
    lib.rn_plan_run.argtypes = [vp, i64p, i32p, vp]
    lib.rn_plan_free.argtypes = [vp]
    lib.rn_plan_free.restype = None
    lib.rn_server_create.argtypes = [vp, C.POINTER(ServerConfig), C.POINTER(vp)]
    lib.rn_server_submit.argtypes = [vp, i32p, C.c_int32, i32p, C.c_int32, C.c_uint32, C.c_int32, i64p]
    lib.rn_server_wait.argtypes = [vp, C.c_int64, vp, C.c_int64, i64p, C.POINTER(C.c_double)]
    lib.rn_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    lib.rn_server_free.argtypes = [vp]
    lib.rn_server_free.restype = None
    lib.rn_objects_graph.argtypes = [vp, C.c_int32, i32p, u32p, C.c_int32, C.POINTER(vp)]
    lib.rn_last_error.restype = C.c_char_p
    lib.rn_version.restype = C.c_char_p
    for name in ("rn_graph_load", "rn_graph_num_vertices", "rn_partition_host", "rn_partition", "rn_graph_renumbered",
                 "rn_dist_join", "rn_kcp_join", "rn_set_tuning", "rn_get_tuning",
                 "rn_set_profiling", "rn_last_stats", "rn_graph_load_many", "rn_graph_count",
                 "rn_graph_size", "rn_join_batch", "rn_autotune", "rn_plan_create", "rn_plan_run",
                 "rn_server_create", "rn_server_submit", "rn_server_wait", "rn_server_get_stats",
                 "rn_objects_graph", "rn_dist_join_noalloc"):
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
    """Graphs resident on the current HIP device (an rn_graph handle).

    A handle holds one graph (``from_graph``) or several (``from_graphs``);
    the single-query calls use graph 0, ``join_batch`` any of them."""

    def __init__(self, row_ptr, col, w):
        self._load([(row_ptr, col, w)])

    def _load(self, csrs):
        lib = load_library()
        keep = [(_host(rp, np.int32)[0], _host(cl, np.int32)[0], _host(ww, np.uint32)[0]) for rp, cl, ww in csrs]
        n = len(keep)
        Vs = np.array([k[0].shape[0] - 1 for k in keep], dtype=np.int32)
        As = np.array([k[1].shape[0] for k in keep], dtype=np.int64)
        ptrs = [(C.c_void_p * n)(*[k[j].ctypes.data for k in keep]) for j in range(3)]
        h = C.c_void_p()
        self._h = None
        _check(lib.rn_graph_load_many(n, Vs.ctypes.data_as(C.POINTER(C.c_int32)),
                                      As.ctypes.data_as(C.POINTER(C.c_int64)), *ptrs, C.byref(h)))
        self._h = h
        self.sizes = [(int(v), int(a)) for v, a in zip(Vs, As)]
        self.V = int(Vs.sum())
        self.A = int(As.sum())
        self._out = None
        self._bout = None

    @classmethod
    def from_graph(cls, g) -> "RoadNetwork":
        return cls(g.row_ptr, g.col, g.w)

    @classmethod
    def from_graphs(cls, graphs) -> "RoadNetwork":
        self = cls.__new__(cls)
        self._load([(g.row_ptr, g.col, g.w) for g in graphs])
        return self

    def with_objects(self, arcs, offsets, graph: int = 0) -> "RoadNetwork":
        """A new handle: graph `graph` with object i (on arc arcs[i], at
        offsets[i] from its tail) inserted as vertex V + i (rn_objects_graph)."""
        lib = load_library()
        a, ap = _host(arcs, np.int32)
        o, op = _host(offsets, np.uint32)
        h = C.c_void_p()
        _check(lib.rn_objects_graph(self._h, int(graph), ap, op, int(a.shape[0]), C.byref(h)))
        V, A = C.c_int32(), C.c_int64()
        _check(lib.rn_graph_size(h, 0, C.byref(V), C.byref(A)))
        net = RoadNetwork.__new__(RoadNetwork)
        net._h, net._out, net._bout = h, None, None
        net.sizes = [(int(V.value), int(A.value))]
        net.V, net.A = int(V.value), int(A.value)
        return net

    @property
    def num_graphs(self) -> int:
        return int(load_library().rn_graph_count(self._h))

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

    def renumbered(self, graph: int = 0) -> bool:
        """Whether rn_partition put the device copy of `graph` in leaf order."""
        return bool(load_library().rn_graph_renumbered(self._h, int(graph)))

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

    def _call(self, fn, R, S, arg, stream, guess):
        import torch
        R, S = self._dev_ids(R), self._dev_ids(S)
        if stream is None:
            stream = torch.cuda.current_stream()
        sptr = C.c_void_p(stream.cuda_stream)
        n = C.c_int64()
        # a first buffer large enough for most calls, so that a call is rarely
        # issued twice (the second time only after RN_ERR_CAPACITY)
        out = self._out_buffer(min(int(guess), R.numel() * S.numel()))
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
        return self._call(load_library().rn_dist_join, R, S, C.c_uint32(int(theta)), stream, 1 << 22)

    def kcp_join(self, R, S, k: int, stream=None):
        """k closest pairs on the device: int32 tensor [n, 3], n = min(k, reachable pairs)."""
        return self._call(load_library().rn_kcp_join, R, S, C.c_int32(int(k)), stream, int(k))

    # -------------------------------------------------------------- batches
    def make_queries(self, specs, keep: list | None = None):
        """rn_query array from dicts {R, S, theta=MAX_DIST, k=0, graph=0, delta=None, hash_log2=0,
        forward=False}.

        R and S become int32 device tensors, appended to ``keep`` (they must stay
        alive while the queries are used)."""
        arr = (Query * len(specs))()
        keep = [] if keep is None else keep
        for i, sp in enumerate(specs):
            R, S = self._dev_ids(sp["R"]), self._dev_ids(sp["S"])
            keep += [R, S]
            d = sp.get("delta")
            arr[i] = Query(R.data_ptr(), S.data_ptr(), R.numel(), S.numel(), int(sp.get("graph", 0)),
                           int(sp.get("k", 0)), int(sp.get("theta", MAX_DIST)),
                           RN_DELTA_DEFAULT if d is None else int(d), int(sp.get("hash_log2", 0)),
                           RN_QUERY_FORWARD if sp.get("forward") else 0)
        return arr, keep

    def _bout_buffer(self, n: int):
        import torch
        if self._bout is None or self._bout.shape[0] < n:
            self._bout = torch.empty((max(n, 1024), 3), dtype=torch.int32, device="cuda")
        return self._bout

    def join_batch(self, queries, stream=None, check: bool = True):
        """Run a batch: returns (pairs tensor [total, 3], offsets int64[nq+1], status int32[nq]).

        ``queries``: an rn_query array (``make_queries``) or a list of dicts.
        Query i's pairs are rows offsets[i]..offsets[i+1].  With ``check`` an
        RN_ERR_ARG from the device raises; otherwise status reports it."""
        import torch
        keep = []
        if not isinstance(queries, C.Array):
            queries, keep = self.make_queries(queries)
        nq = len(queries)
        if stream is None:
            stream = torch.cuda.current_stream()
        sptr = C.c_void_p(stream.cuda_stream)
        off = np.zeros(nq + 1, dtype=np.int64)
        status = np.zeros(nq, dtype=np.int32)
        lib = load_library()
        out = self._bout_buffer(0)

        def call(o):
            return lib.rn_join_batch(self._h, queries, nq, C.c_void_p(o.data_ptr()), o.shape[0],
                                     off.ctypes.data_as(C.POINTER(C.c_int64)),
                                     status.ctypes.data_as(C.POINTER(C.c_int32)), sptr)
        st = call(out)
        if st == RN_ERR_CAPACITY and off[nq] > out.shape[0]:
            out = self._bout_buffer(int(off[nq]))
            st = call(out)
        if st != RN_OK and not (st == RN_ERR_ARG and not check and status.any()):
            _check(st, int(off[nq]))
        del keep
        return out[: int(off[nq])], off, status

    def autotune(self, queries, sample: int = 256, stream=None):
        """Pick delta / hash_log2 per query in place (rn_autotune)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(load_library().rn_autotune(self._h, queries, len(queries), int(sample),
                                          C.c_void_p(stream.cuda_stream)))
        return queries

    def plan(self, queries, cap: int | None = None, stream=None) -> "Plan":
        """Capture a batch into a HIP graph (see Plan)."""
        return Plan(self, queries, cap, stream)


class Plan:
    """A batch captured once into a HIP graph and replayed by ``run``.

    The plan keeps the query array (and the device R, S tensors it points to)
    and an output buffer of ``cap`` pairs (the batch's size when None)."""

    def __init__(self, net: RoadNetwork, queries, cap: int | None = None, stream=None):
        import torch
        self.net, self.queries = net, queries
        if cap is None:
            _, off, _ = net.join_batch(queries, stream=stream, check=False)
            cap = int(off[-1]) + 1024
        self.out = torch.empty((max(int(cap), 1), 3), dtype=torch.int32, device="cuda")
        if stream is None:
            stream = torch.cuda.current_stream()
        h = C.c_void_p()
        self._h = None
        _check(load_library().rn_plan_create(net._h, queries, len(queries), C.c_void_p(self.out.data_ptr()),
                                             int(cap), C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h
        # what every run passes, built once (a replay is a few hundred microseconds)
        self._stream = C.c_void_p(stream.cuda_stream)
        self._off = np.zeros(len(queries) + 1, dtype=np.int64)
        self._status = np.zeros(len(queries), dtype=np.int32)
        self._offp = self._off.ctypes.data_as(C.POINTER(C.c_int64))
        self._statusp = self._status.ctypes.data_as(C.POINTER(C.c_int32))
        self._run = load_library().rn_plan_run

    def run(self, stream=None, check: bool = True):
        """Replay on ``stream`` (default: the stream the plan was created on):
        returns (pairs tensor view, offsets, status) as join_batch."""
        sp = self._stream if stream is None else C.c_void_p(stream.cuda_stream)
        st = self._run(self._h, self._offp, self._statusp, sp)
        off, status = self._off.copy(), self._status.copy()
        n = int(off[-1])
        if st != RN_OK and not (st == RN_ERR_ARG and not check and status.any()):
            _check(st, n)
        return self.out[:n], off, status

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().rn_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_batch(out, off) -> list[np.ndarray]:
    """Pairs tensor + offsets -> one structured numpy array per query."""
    a = pairs_to_numpy(out)
    return [a[int(off[i]):int(off[i + 1])] for i in range(len(off) - 1)]


class Server:
    """A request server on one graph of a handle (rn_server_*): submit host
    node sets, wait for host results; batching and overlap happen inside."""

    def __init__(self, net: RoadNetwork, graph: int = 0, lanes: int = 2, max_batch: int = 8,
                 global_slots: int = 128, hbm_budget: int = 8 << 30, heavy_lane: bool = True):
        self.net = net
        cfg = ServerConfig(int(graph), int(lanes), int(max_batch), int(global_slots), int(hbm_budget),
                           1 if heavy_lane else 0, 0)
        h = C.c_void_p()
        self._h = None
        _check(load_library().rn_server_create(net._h, C.byref(cfg), C.byref(h)))
        self._h = h

    def submit(self, R, S, theta: int = MAX_DIST, k: int = 0) -> int:
        Rh, Rp = _host(R, np.int32)
        Sh, Sp = _host(S, np.int32)
        rid = C.c_int64()
        _check(load_library().rn_server_submit(self._h, Rp, Rh.shape[0], Sp, Sh.shape[0], int(theta), int(k),
                                               C.byref(rid)))
        return rid.value

    def wait(self, rid: int, guess: int = 4096):
        """Block until request rid is answered: (structured pair array, latency in ms)."""
        lib = load_library()
        n, lat = C.c_int64(), C.c_double()
        out = np.empty(max(int(guess), 1), dtype=PAIR_DTYPE)
        st = lib.rn_server_wait(self._h, int(rid), out.ctypes.data, out.shape[0], C.byref(n), C.byref(lat))
        if st == RN_ERR_CAPACITY:
            out = np.empty(n.value, dtype=PAIR_DTYPE)
            st = lib.rn_server_wait(self._h, int(rid), out.ctypes.data, out.shape[0], C.byref(n), C.byref(lat))
        _check(st, n.value)
        return out[: n.value], lat.value

    def stats(self) -> dict:
        s = ServerStats()
        _check(load_library().rn_server_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().rn_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
