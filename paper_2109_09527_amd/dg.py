"""Python binding of libdg (the C boundary declared in include/dg.h).

Argument marshalling only: every step runs in the HIP library.  torch
supplies device buffers and the current HIP stream.  Importing this module
loads paper_2109_09527_amd/libdg.so and raises if it is not built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from .synth import OP_DTYPE

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdg.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run paper_2109_09527_amd/build.py")
lib = ctypes.CDLL(_LIB_PATH)

EPOCH_LATEST = 0xFFFFFFFF
OK, E_INVALID_ARG, E_OUT_OF_MEMORY, E_VERTEX_RANGE, E_WEIGHT_RANGE = 0, -1, -2, -3, -4
E_EPOCH_RETIRED, E_SOURCE_ABSENT, E_OVERFLOW, E_HIP, E_BUSY, E_UNIMPLEMENTED = -5, -6, -7, -8, -9, -10
UNDIRECTED = 1
Q_BFS, Q_SSSP, Q_BC = 0, 1, 2

_P = ctypes.c_void_p
_u32, _i32, _u64 = ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64


class Config(ctypes.Structure):
    _fields_ = [("v_capacity", _u32), ("flags", _u32), ("w_max", _i32), ("max_resident_epochs", _u32),
                ("edge_capacity", _u64), ("mem_budget", _u64)]


class Tuning(ctypes.Structure):
    _fields_ = [("chunk_buckets", _u32), ("sssp_delta", _u32), ("alpha", _u32), ("beta", _u32),
                ("batch_groups", _u32), ("batch_delta", _u32), ("batch_gang", _u32)]


class Query(ctypes.Structure):
    _fields_ = [("kind", _u32), ("src", _u32), ("epoch", _u32), ("k", _u32), ("srcs", _P), ("out", _P)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mem_budget", _u64), ("max_inflight", _u32), ("max_batch", _u32), ("query_lanes", _u32),
                ("log_ops", _u32), ("bfs_rounds", _u32), ("sssp_rounds", _u32)]


class LogRecord(ctypes.Structure):
    _fields_ = [("ticket", _u64), ("kind", _i32), ("status", _i32), ("epoch", _u32), ("n", _u32), ("off", _u64),
                ("t_arrive_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", _u64), ("updates", _u64), ("queries", _u64), ("ops_applied", _u64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("p50_query_ms", ctypes.c_double), ("p99_query_ms", ctypes.c_double),
                ("p50_update_ms", ctypes.c_double), ("p99_update_ms", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("edges_traversed", _u64), ("joined_running", _u64)]


def _sig(name, res, *args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("dg_create", _i32, ctypes.POINTER(Config), ctypes.POINTER(_P))
_sig("dg_destroy", _i32, _P)
_sig("dg_last_error", ctypes.c_char_p, _P)
_sig("dg_latest_epoch", _u32, _P)
_sig("dg_apply_batch", _i32, _P, _P, _u64, _P, ctypes.POINTER(_u32), _P)
for _n in ("dg_add_vertex", "dg_remove_vertex", "dg_contains_vertex"):
    _sig(_n, _i32, _P, _u32, _P, ctypes.POINTER(_u32))
_sig("dg_add_edge", _i32, _P, _u32, _u32, _i32, _P, ctypes.POINTER(_u32))
_sig("dg_remove_edge", _i32, _P, _u32, _u32, _P, ctypes.POINTER(_u32))
_sig("dg_contains_edge", _i32, _P, _u32, _u32, _P, ctypes.POINTER(_u32))
_sig("dg_snapshot_acquire", _i32, _P, _u32, ctypes.POINTER(_u32))
_sig("dg_snapshot_release", _i32, _P, _u32)
_sig("dg_compact", _i32, _P, _P)
_sig("dg_bfs", _i32, _P, _u32, _u32, _P, _P)
_sig("dg_bfs_noalloc", _i32, _P, _u32, _u32, _P, _P)
NOALLOC_SCRATCH_BYTES = 96 << 20   # DG_NOALLOC_SCRATCH_BYTES
_sig("dg_sssp", _i32, _P, _u32, _u32, _P, _P)
_sig("dg_bc", _i32, _P, _u32, _P, _u32, _P, _P)
for _n in ("dg_pagerank", "dg_pagerank_nosync"):
    _sig(_n, _i32, _P, _u32, ctypes.c_double, ctypes.c_double, _u32, _P, ctypes.POINTER(_u32),
         ctypes.POINTER(ctypes.c_double), _P)


_sig("dg_scc", _i32, _P, _u32, _P, ctypes.POINTER(_u32), _P)
_sig("dg_diameter", _i32, _P, _u32, ctypes.POINTER(_u32), _P)
_sig("dg_maxflow", _i32, _P, _u32, _u32, _u32, ctypes.POINTER(ctypes.c_int64), _P)
_sig("dg_dfs", _i32, _P, _u32, _u32, _P, _P, ctypes.POINTER(_u32), _P)


class PageRankOpts(ctypes.Structure):
    _fields_ = [("damping", ctypes.c_double), ("threshold", ctypes.c_double), ("freeze_below", ctypes.c_double),
                ("max_iters", _u32), ("nosync", ctypes.c_int)]


_sig("dg_pagerank_ex", _i32, _P, _u32, ctypes.POINTER(PageRankOpts), _P, ctypes.POINTER(_u32),
     ctypes.POINTER(ctypes.c_double), _P)
_sig("dg_query_batch", _i32, _P, _P, _u32, _P, _P)
_sig("dg_get_tuning", _i32, _P, ctypes.POINTER(Tuning))
_sig("dg_set_tuning", _i32, _P, ctypes.POINTER(Tuning))
_sig("dg_autotune", _i32, _P, _u32, ctypes.POINTER(Tuning), _P)
_sig("dg_stats", _i32, _P, _u32, ctypes.POINTER(_u64), ctypes.POINTER(_u64), _P)
_sig("dg_out_degrees", _i32, _P, _u32, _P, _P)
class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", _u64), ("total_ms", ctypes.c_double), ("arcs", _u64)]


_sig("dg_profile_enable", _i32, _P, ctypes.c_int)
_sig("dg_profile_read", _i32, _P, _P, _u32, ctypes.POINTER(_u32), ctypes.c_int)
_sig("dg_server_start", _i32, _P, ctypes.POINTER(ServerConfig), ctypes.POINTER(_P))
_sig("dg_server_stop", _i32, _P)
_sig("dg_server_submit_update", _i32, _P, _P, _u64, ctypes.POINTER(_u64))
_sig("dg_server_submit_query", _i32, _P, _u32, _P, _u32, ctypes.POINTER(_u64))
_sig("dg_server_poll", _i32, _P, _u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i32), ctypes.POINTER(_u32),
     ctypes.POINTER(ctypes.c_double))
_sig("dg_server_take", _i32, _P, _u64, _P, _u64)
_sig("dg_server_drain", _i32, _P)
_sig("dg_server_log", _i32, _P, _P, _u64, ctypes.POINTER(_u64), _P, _u64, ctypes.POINTER(_u64), _P, _u64,
     ctypes.POINTER(_u64))
_sig("dg_server_get_stats", _i32, _P, ctypes.POINTER(ServerStats))

EXPORTED = [n for n in dir(lib) if n.startswith("dg_")]


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dg status {status}: {msg}")
        self.status = status


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(x):
    if isinstance(x, torch.Tensor):
        return ctypes.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(ctypes.c_void_p)
    return x


def ops_to_device(ops: np.ndarray, device="cuda") -> torch.Tensor:
    """Copy a host op array (synth.OP_DTYPE) to a device tensor of the same bytes."""
    a = np.ascontiguousarray(ops).view(np.int32).reshape(-1, 4)
    return torch.from_numpy(a.copy()).to(device)


class Graph:
    """One dynamic graph on the current HIP device."""

    def __init__(self, v_capacity: int, undirected: bool = False, w_max: int = 255,
                 max_resident_epochs: int = 8, edge_capacity: int = 0, mem_budget: int = 0):
        cfg = Config(v_capacity, UNDIRECTED if undirected else 0, w_max, max_resident_epochs,
                     edge_capacity, mem_budget)
        h = _P()
        rc = lib.dg_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != OK:
            raise DGError(rc, lib.dg_last_error(None).decode())
        self.h = h
        self.n = v_capacity
        self.undirected = undirected

    def close(self):
        if getattr(self, "h", None):
            lib.dg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise DGError(rc, lib.dg_last_error(self.h).decode())

    @property
    def epoch(self) -> int:
        return int(lib.dg_latest_epoch(self.h))

    def try_apply(self, ops, results=None):
        """Returns (status, results, epoch) without raising."""
        if isinstance(ops, np.ndarray):
            ops = np.ascontiguousarray(ops.astype(OP_DTYPE, copy=False))
            n = len(ops)
        else:
            n = ops.numel() // 4
        if results is None:
            results = np.zeros(n, dtype=np.uint8)
        ep = _u32()
        rc = lib.dg_apply_batch(self.h, _ptr(ops), n, _ptr(results), ctypes.byref(ep), _stream())
        return rc, results, int(ep.value)

    def apply(self, ops, results=None):
        rc, res, ep = self.try_apply(ops, results)
        self._check(rc)
        return res, ep

    def _single(self, fn, *args):
        r = ctypes.c_uint8()
        ep = _u32()
        self._check(fn(self.h, *args, ctypes.byref(r), ctypes.byref(ep)))
        return int(r.value), int(ep.value)

    def add_vertex(self, v):
        return self._single(lib.dg_add_vertex, v)

    def remove_vertex(self, v):
        return self._single(lib.dg_remove_vertex, v)

    def contains_vertex(self, v):
        return self._single(lib.dg_contains_vertex, v)

    def add_edge(self, u, v, w):
        return self._single(lib.dg_add_edge, u, v, w)

    def remove_edge(self, u, v):
        return self._single(lib.dg_remove_edge, u, v)

    def contains_edge(self, u, v):
        return self._single(lib.dg_contains_edge, u, v)

    def acquire(self, epoch=EPOCH_LATEST) -> int:
        e = _u32()
        self._check(lib.dg_snapshot_acquire(self.h, epoch, ctypes.byref(e)))
        return int(e.value)

    def release(self, epoch: int):
        self._check(lib.dg_snapshot_release(self.h, epoch))

    def compact(self):
        self._check(lib.dg_compact(self.h, _stream()))

    def try_bfs(self, src, epoch=EPOCH_LATEST, out=None):
        out = torch.empty(self.n, dtype=torch.int32, device="cuda") if out is None else out
        return lib.dg_bfs(self.h, epoch, src, _ptr(out), _stream()), out

    def bfs(self, src, epoch=EPOCH_LATEST, out=None) -> torch.Tensor:
        rc, out = self.try_bfs(src, epoch, out)
        self._check(rc)
        return out

    def try_bfs_noalloc(self, src, epoch=EPOCH_LATEST, out=None):
        out = torch.empty(self.n, dtype=torch.int32, device="cuda") if out is None else out
        return lib.dg_bfs_noalloc(self.h, epoch, src, _ptr(out), _stream()), out

    def bfs_noalloc(self, src, epoch=EPOCH_LATEST, out=None) -> torch.Tensor:
        rc, out = self.try_bfs_noalloc(src, epoch, out)
        self._check(rc)
        return out

    def try_sssp(self, src, epoch=EPOCH_LATEST, out=None):
        out = torch.empty(self.n, dtype=torch.int32, device="cuda") if out is None else out
        return lib.dg_sssp(self.h, epoch, src, _ptr(out), _stream()), out

    def sssp(self, src, epoch=EPOCH_LATEST, out=None) -> torch.Tensor:
        rc, out = self.try_sssp(src, epoch, out)
        self._check(rc)
        return out

    def try_bc(self, srcs, epoch=EPOCH_LATEST, out=None):
        S = np.ascontiguousarray(np.asarray(srcs, dtype=np.uint32))
        out = torch.empty(self.n, dtype=torch.float64, device="cuda") if out is None else out
        return lib.dg_bc(self.h, epoch, _ptr(S), len(S), _ptr(out), _stream()), out

    def bc(self, srcs, epoch=EPOCH_LATEST, out=None) -> torch.Tensor:
        rc, out = self.try_bc(srcs, epoch, out)
        self._check(rc)
        return out

    def try_scc(self, epoch=EPOCH_LATEST, out=None):
        """(status, comp tensor int32, number of components)."""
        out = torch.empty(self.n, dtype=torch.int32, device="cuda") if out is None else out
        nc = _u32()
        rc = lib.dg_scc(self.h, epoch, _ptr(out), ctypes.byref(nc), _stream())
        return rc, out, int(nc.value)

    def scc(self, epoch=EPOCH_LATEST, out=None):
        """(comp tensor, number of components); raises on a failed call."""
        rc, out, nc = self.try_scc(epoch, out)
        self._check(rc)
        return out, nc

    def diameter(self, epoch=EPOCH_LATEST) -> int:
        """Largest hop distance over reachable ordered pairs of live vertices."""
        d = _u32()
        self._check(lib.dg_diameter(self.h, epoch, ctypes.byref(d), _stream()))
        return int(d.value)

    def try_maxflow(self, s, t, epoch=EPOCH_LATEST):
        """(status, maximum s-t flow with arc weights as capacities)."""
        f = ctypes.c_int64()
        rc = lib.dg_maxflow(self.h, epoch, int(s), int(t), ctypes.byref(f), _stream())
        return rc, int(f.value)

    def maxflow(self, s, t, epoch=EPOCH_LATEST) -> int:
        rc, f = self.try_maxflow(s, t, epoch)
        self._check(rc)
        return f

    def try_dfs(self, s, epoch=EPOCH_LATEST, disc=None, parent=None):
        """(status, disc tensor int32, parent tensor int32, vertices reached):
        depth-first search from s taking neighbours in ascending id order."""
        disc = torch.empty(self.n, dtype=torch.int32, device="cuda") if disc is None else disc
        parent = torch.empty(self.n, dtype=torch.int32, device="cuda") if parent is None else parent
        nr = _u32()
        rc = lib.dg_dfs(self.h, epoch, int(s), _ptr(disc), _ptr(parent), ctypes.byref(nr), _stream())
        return rc, disc, parent, int(nr.value)

    def dfs(self, s, epoch=EPOCH_LATEST, disc=None, parent=None):
        """(disc, parent, vertices reached); raises on a failed call."""
        rc, disc, parent, nr = self.try_dfs(s, epoch, disc, parent)
        self._check(rc)
        return disc, parent, nr

    def try_pagerank(self, epoch=EPOCH_LATEST, damping=0.85, threshold=1e-16, max_iters=10000, out=None,
                     nosync=False, freeze_below=None):
        """(status, pr tensor, iterations, last iteration's largest change);
        nosync: the barrier-free form (iterations = most sweeps of a workgroup);
        freeze_below: loop perforation (dg_pagerank_ex)."""
        out = torch.empty(self.n, dtype=torch.float64, device="cuda") if out is None else out
        it = _u32()
        ch = ctypes.c_double()
        if freeze_below is None:
            fn = lib.dg_pagerank_nosync if nosync else lib.dg_pagerank
            rc = fn(self.h, epoch, float(damping), float(threshold), int(max_iters), _ptr(out), ctypes.byref(it),
                    ctypes.byref(ch), _stream())
        else:
            o = PageRankOpts(float(damping), float(threshold), float(freeze_below), int(max_iters), int(nosync))
            rc = lib.dg_pagerank_ex(self.h, epoch, ctypes.byref(o), _ptr(out), ctypes.byref(it), ctypes.byref(ch),
                                    _stream())
        return rc, out, int(it.value), float(ch.value)

    def pagerank(self, epoch=EPOCH_LATEST, damping=0.85, threshold=1e-16, max_iters=10000, out=None,
                 nosync=False, freeze_below=None):
        """(pr tensor, iterations, last change); raises on a failed call."""
        rc, out, it, ch = self.try_pagerank(epoch, damping, threshold, max_iters, out, nosync, freeze_below)
        self._check(rc)
        return out, it, ch

    def query_batch(self, queries):
        """queries: list of (kind, epoch, src_or_srcs, out_tensor).  Returns
        the per-query status list (the call status raises on failure)."""
        nq = len(queries)
        arr = (Query * max(nq, 1))()
        keep = []
        for i, (kind, ep, src, out) in enumerate(queries):
            if kind == Q_BC:
                S = np.ascontiguousarray(np.asarray(src, dtype=np.uint32))
                keep.append(S)
                arr[i] = Query(kind, 0, ep, len(S), S.ctypes.data, out.data_ptr())
            else:
                arr[i] = Query(kind, int(src), ep, 0, None, out.data_ptr())
        st = (_i32 * max(nq, 1))()
        self._check(lib.dg_query_batch(self.h, arr, nq, st, _stream()))
        return [int(st[i]) for i in range(nq)]

    def stats(self, epoch=EPOCH_LATEST):
        nv, na = _u64(), _u64()
        self._check(lib.dg_stats(self.h, epoch, ctypes.byref(nv), ctypes.byref(na), _stream()))
        return int(nv.value), int(na.value)

    def out_degrees(self, epoch=EPOCH_LATEST) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self._check(lib.dg_out_degrees(self.h, epoch, _ptr(out), _stream()))
        return out

    def profile(self, on: bool):
        self._check(lib.dg_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, reset: bool = True) -> dict:
        """{family: {"launches", "total_ms", "arcs"}} for kernel families with launches."""
        arr = (KernelStat * 32)()
        n = _u32()
        self._check(lib.dg_profile_read(self.h, arr, 32, ctypes.byref(n), 1 if reset else 0))
        out = {}
        for i in range(n.value):
            k = arr[i]
            if k.launches:
                out[k.name.decode()] = {"launches": int(k.launches), "total_ms": float(k.total_ms),
                                        "arcs": int(k.arcs)}
        return out

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(lib.dg_get_tuning(self.h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = Tuning(**cur)
        self._check(lib.dg_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, seed=0) -> dict:
        t = Tuning()
        self._check(lib.dg_autotune(self.h, seed, ctypes.byref(t), _stream()))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}


class Server:
    """Serving loop over a Graph (dg_server_*)."""

    def __init__(self, graph: Graph, mem_budget=8 << 30, max_inflight=64, max_batch=32, query_lanes=1,
                 log_ops=False, bfs_rounds=False, sssp_rounds=False):
        cfg = ServerConfig(mem_budget, max_inflight, max_batch, query_lanes, 1 if log_ops else 0,
                           1 if bfs_rounds else 0, 1 if sssp_rounds else 0)
        h = _P()
        rc = lib.dg_server_start(graph.h, ctypes.byref(cfg), ctypes.byref(h))
        if rc != OK:
            raise DGError(rc, lib.dg_last_error(graph.h).decode())
        self.h = h
        self.g = graph

    def submit_update(self, ops: np.ndarray) -> int:
        ops = np.ascontiguousarray(ops.astype(OP_DTYPE, copy=False))
        t = _u64()
        self.g._check(lib.dg_server_submit_update(self.h, _ptr(ops), len(ops), ctypes.byref(t)))
        return int(t.value)

    def submit_query(self, kind: int, srcs) -> int:
        S = np.ascontiguousarray(np.atleast_1d(np.asarray(srcs, dtype=np.uint32)))
        t = _u64()
        self.g._check(lib.dg_server_submit_query(self.h, kind, _ptr(S), len(S), ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int):
        done, st, ep, lat = ctypes.c_int(), _i32(), _u32(), ctypes.c_double()
        self.g._check(lib.dg_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(ep),
                                         ctypes.byref(lat)))
        return bool(done.value), int(st.value), int(ep.value), float(lat.value)

    def take(self, ticket: int, out: np.ndarray):
        self.g._check(lib.dg_server_take(self.h, ticket, _ptr(out), out.nbytes))
        return out

    def drain(self):
        self.g._check(lib.dg_server_drain(self.h))

    def log(self):
        """The library's log in linearization order: a list of dicts with
        ticket, kind ("update" / "bfs" / "sssp" / "bc"), status, epoch and
        ops (updates, when kept) or srcs (queries)."""
        nr, no, ns = _u64(), _u64(), _u64()
        self.g._check(lib.dg_server_log(self.h, None, 0, ctypes.byref(nr), None, 0, ctypes.byref(no), None, 0,
                                        ctypes.byref(ns)))
        recs = (LogRecord * max(1, nr.value))()
        ops = np.zeros(max(1, no.value), dtype=OP_DTYPE)
        srcs = np.zeros(max(1, ns.value), dtype=np.uint32)
        self.g._check(lib.dg_server_log(self.h, recs, nr.value, ctypes.byref(nr), _ptr(ops), no.value,
                                        ctypes.byref(no), _ptr(srcs), ns.value, ctypes.byref(ns)))
        names = {-1: "update", Q_BFS: "bfs", Q_SSSP: "sssp", Q_BC: "bc"}
        out = []
        for i in range(nr.value):
            r = recs[i]
            d = {"ticket": int(r.ticket), "kind": names[r.kind], "status": int(r.status), "epoch": int(r.epoch),
                 "t_arrive_ms": r.t_arrive_ms, "t_done_ms": r.t_done_ms}
            if r.kind < 0:
                d["ops"] = None if r.off == 0xFFFFFFFFFFFFFFFF else ops[r.off:r.off + r.n].copy()
            else:
                d["srcs"] = [int(x) for x in srcs[r.off:r.off + r.n]]
            out.append(d)
        return out

    def stats(self) -> dict:
        s = ServerStats()
        self.g._check(lib.dg_server_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def stop(self):
        if getattr(self, "h", None):
            lib.dg_server_stop(self.h)
            self.h = None
