"""Python handle on the sequential CPU oracle (dg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg.  The product package never imports it.

`build()` compiles the C source with gcc; `Oracle` wraps one oracle graph.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "dg_oracle.c")
_LIB = os.path.join(_DIR, "libdg_oracle.so")

OK, E_INVALID_ARG, E_OOM, E_VERTEX_RANGE, E_WEIGHT_RANGE = 0, -1, -2, -3, -4
E_SOURCE_ABSENT, E_OVERFLOW = -6, -7

_lib = None


def build() -> str:
    """Compile the oracle into oracle/libdg_oracle.so (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    u32, i32, u64 = ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [u32, ctypes.c_int, i32]
    lib.orc_destroy.argtypes = [P]
    lib.orc_epoch.restype = u32
    lib.orc_epoch.argtypes = [P]
    lib.orc_apply.restype = ctypes.c_int
    lib.orc_apply.argtypes = [P, P, u64, P]
    for f in (lib.orc_bfs, lib.orc_sssp):
        f.restype = ctypes.c_int
        f.argtypes = [P, u32, P]
    lib.orc_bc.restype = ctypes.c_int
    lib.orc_bc.argtypes = [P, P, u32, P]
    lib.orc_counts.argtypes = [P, P, P]
    lib.orc_alive.restype = ctypes.c_int
    lib.orc_alive.argtypes = [P, u32]
    lib.orc_edge.restype = ctypes.c_int
    lib.orc_edge.argtypes = [P, u32, u32, P]
    lib.orc_n_keys.restype = u64
    lib.orc_n_keys.argtypes = [P]
    lib.orc_export.restype = u64
    lib.orc_export.argtypes = [P, P, P, P]
    lib.orc_out_degree.restype = u32
    lib.orc_out_degree.argtypes = [P, u32]
    lib.orc_pagerank.restype = ctypes.c_int
    lib.orc_pagerank.argtypes = [P, ctypes.c_double, ctypes.c_double, u32, P, P, P]
    lib.orc_scc.restype = ctypes.c_int
    lib.orc_scc.argtypes = [P, P]
    lib.orc_diameter.restype = ctypes.c_int
    lib.orc_diameter.argtypes = [P, P]
    lib.orc_maxflow.restype = ctypes.c_int
    lib.orc_maxflow.argtypes = [P, u32, u32, P]
    lib.orc_dfs.restype = ctypes.c_int
    lib.orc_dfs.argtypes = [P, u32, P, P]
    lib.orc_pagerank_perforated.restype = ctypes.c_int
    lib.orc_pagerank_perforated.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, u32, P, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """One sequential graph: ops applied in index order, queries on the
    current state (the snapshot of the latest epoch)."""

    def __init__(self, n_vertices: int, undirected: bool = False, w_max: int = 255):
        self.lib = _load()
        self.n = int(n_vertices)
        self.undirected = bool(undirected)
        self.h = self.lib.orc_create(self.n, 1 if undirected else 0, int(w_max))
        if not self.h:
            raise ValueError("oracle: invalid configuration")

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    __del__ = close

    @property
    def epoch(self) -> int:
        return int(self.lib.orc_epoch(self.h))

    def apply(self, ops: np.ndarray):
        """Returns (status, results uint8[n])."""
        ops = np.ascontiguousarray(ops)
        res = np.zeros(len(ops), dtype=np.uint8)
        rc = self.lib.orc_apply(self.h, _ptr(ops), len(ops), _ptr(res))
        return rc, res

    def bfs(self, s: int):
        d = np.empty(self.n, dtype=np.int32)
        rc = self.lib.orc_bfs(self.h, int(s), _ptr(d))
        return rc, d

    def sssp(self, s: int):
        d = np.empty(self.n, dtype=np.int32)
        rc = self.lib.orc_sssp(self.h, int(s), _ptr(d))
        return rc, d

    def bc(self, S):
        S = np.ascontiguousarray(np.asarray(S, dtype=np.uint32))
        out = np.zeros(self.n, dtype=np.float64)
        rc = self.lib.orc_bc(self.h, _ptr(S), len(S), _ptr(out))
        return rc, out

    def counts(self):
        nv = ctypes.c_uint64()
        na = ctypes.c_uint64()
        self.lib.orc_counts(self.h, ctypes.byref(nv), ctypes.byref(na))
        return nv.value, na.value

    def alive(self, v: int) -> bool:
        return bool(self.lib.orc_alive(self.h, int(v)))

    def edge(self, u: int, v: int):
        w = ctypes.c_int32()
        ok = self.lib.orc_edge(self.h, int(u), int(v), ctypes.byref(w))
        return (True, w.value) if ok else (False, 0)

    def out_degree(self, v: int) -> int:
        return int(self.lib.orc_out_degree(self.h, int(v)))

    def scc(self):
        """(status, comp[n] int32): smallest id of each live vertex's strongly
        connected component, -1 for vertices that are not live."""
        out = np.empty(self.n, dtype=np.int32)
        rc = self.lib.orc_scc(self.h, _ptr(out))
        return rc, out

    def diameter(self):
        """(status, largest hop distance between live vertices u, v with v
        reachable from u)."""
        d = ctypes.c_uint32()
        rc = self.lib.orc_diameter(self.h, ctypes.byref(d))
        return rc, d.value

    def maxflow(self, s: int, t: int):
        """(status, maximum s-t flow with arc weights as capacities)."""
        f = ctypes.c_int64()
        rc = self.lib.orc_maxflow(self.h, int(s), int(t), ctypes.byref(f))
        return rc, f.value

    def dfs(self, s: int):
        """(status, disc[n] int32, parent[n] int32): depth-first search from s
        taking out-neighbours in ascending id order; disc = preorder position,
        parent = discovering vertex, -1 where not reached (and parent[s])."""
        disc = np.empty(self.n, dtype=np.int32)
        par = np.empty(self.n, dtype=np.int32)
        rc = self.lib.orc_dfs(self.h, int(s), _ptr(disc), _ptr(par))
        return rc, disc, par

    def pagerank(self, damping=0.85, threshold=1e-16, max_iters=10000, freeze_below=None):
        """(status, pr[n] float64, iterations, last iteration's largest change);
        freeze_below: loop perforation (Alg. 5) below that change."""
        out = np.zeros(self.n, dtype=np.float64)
        it = ctypes.c_uint32()
        ch = ctypes.c_double()
        if freeze_below is None:
            rc = self.lib.orc_pagerank(self.h, float(damping), float(threshold), int(max_iters), _ptr(out),
                                       ctypes.byref(it), ctypes.byref(ch))
        else:
            rc = self.lib.orc_pagerank_perforated(self.h, float(damping), float(threshold), float(freeze_below),
                                                  int(max_iters), _ptr(out), ctypes.byref(it), ctypes.byref(ch))
        return rc, out, it.value, ch.value

    def edges(self):
        """All stored edge keys as (u, v, w) arrays (undirected: u <= v)."""
        k = int(self.lib.orc_n_keys(self.h))
        u = np.empty(k, np.uint32)
        v = np.empty(k, np.uint32)
        w = np.empty(k, np.int32)
        got = self.lib.orc_export(self.h, _ptr(u), _ptr(v), _ptr(w))
        assert got == k
        return u, v, w
