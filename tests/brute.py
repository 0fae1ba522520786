"""Independent brute-force models used to pin the oracle.

None of this is the oracle's algorithm: the ADT is a dense boolean adjacency
matrix, distances come from boolean matrix powers / Warshall closure /
Bellman-Ford relaxation rounds, and betweenness from all-pairs shortest-path
counts read off integer matrix powers (sigma_st = (A^d)[s, t] at the first
d with a non-zero entry), combined with the pair-dependency definition
delta_st(v) = sigma_sv * sigma_vt / sigma_st when d(s,v) + d(v,t) = d(s,t).
"""
from __future__ import annotations

import numpy as np

from paper_2109_09527_amd.synth import ADDV, REMV, HASV, ADDE, REME, HASE


class MatrixModel:
    """Dense model of the graph ADT: alive[n], A[n, n] (arc present), W[n, n]."""

    def __init__(self, n: int, undirected: bool = False):
        self.n = n
        self.und = undirected
        self.alive = np.zeros(n, dtype=bool)
        self.A = np.zeros((n, n), dtype=bool)
        self.W = np.zeros((n, n), dtype=np.int64)

    def _set(self, u, v, present, w=0):
        self.A[u, v] = present
        self.W[u, v] = w if present else 0
        if self.und:
            self.A[v, u] = present
            self.W[v, u] = w if present else 0

    def apply(self, ops) -> np.ndarray:
        res = np.zeros(len(ops), dtype=np.uint8)
        for i, (t, u, v, w) in enumerate(zip(ops["type"].tolist(), ops["u"].tolist(),
                                              ops["v"].tolist(), ops["w"].tolist())):
            if t == ADDV:
                res[i] = 0 if self.alive[u] else 1
                self.alive[u] = True
            elif t == REMV:
                if self.alive[u]:
                    self.A[u, :] = False
                    self.A[:, u] = False
                    self.W[u, :] = 0
                    self.W[:, u] = 0
                    self.alive[u] = False
                    res[i] = 1
            elif t == HASV:
                res[i] = 1 if self.alive[u] else 0
            else:
                if not (self.alive[u] and self.alive[v]):
                    res[i] = 2
                elif t == ADDE:
                    if self.A[u, v]:
                        res[i] = 0
                    else:
                        self._set(u, v, True, w)
                        res[i] = 1
                elif t == REME:
                    res[i] = 1 if self.A[u, v] else 0
                    self._set(u, v, False)
                elif t == HASE:
                    res[i] = 1 if self.A[u, v] else 0
        return res

    def n_arcs(self) -> int:
        return int(self.A.sum())


def bfs_by_powers(A: np.ndarray, s: int) -> np.ndarray:
    """dist[t] = smallest k with (A^k)[s, t] true (boolean products)."""
    n = A.shape[0]
    dist = np.full(n, -1, dtype=np.int64)
    reach = np.zeros(n, dtype=bool)
    reach[s] = True
    dist[s] = 0
    Ai = A.astype(np.int64)
    for k in range(1, n + 1):
        nxt = (reach.astype(np.int64) @ Ai) > 0
        new = nxt & (dist < 0)
        if not new.any():
            break
        dist[new] = k
        reach = new
    return dist


def warshall(A: np.ndarray) -> np.ndarray:
    """Transitive closure (paths of length >= 1) by Warshall's algorithm."""
    R = A.copy()
    for k in range(A.shape[0]):
        R = R | (R[:, k:k + 1] & R[k:k + 1, :])
    return R


def bellman_ford(A: np.ndarray, W: np.ndarray, s: int) -> np.ndarray:
    """n-1 rounds of relaxing every arc; -1 where unreachable."""
    n = A.shape[0]
    INF = np.iinfo(np.int64).max // 4
    d = np.full(n, INF, dtype=np.int64)
    d[s] = 0
    us, vs = np.nonzero(A)
    ws = W[us, vs]
    for _ in range(max(n - 1, 1)):
        cand = d[us] + ws
        nd = d.copy()
        np.minimum.at(nd, vs, np.where(d[us] < INF, cand, INF))
        if np.array_equal(nd, d):
            break
        d = nd
    return np.where(d >= INF, -1, d)


def all_pairs_counts(A: np.ndarray):
    """(dist, sigma) for every pair from integer matrix powers A^k (object
    dtype so counts never overflow).  dist[s, s] = 0, sigma[s, s] = 1."""
    n = A.shape[0]
    dist = np.full((n, n), -1, dtype=np.int64)
    sigma = np.zeros((n, n), dtype=object)
    Ao = A.astype(object)
    P = np.eye(n, dtype=object)   # A^0
    np.fill_diagonal(dist, 0)
    for i in range(n):
        sigma[i, i] = 1
    for k in range(1, n):
        P = P.dot(Ao)
        hit = (P != 0) & (dist < 0)
        if not hit.any():
            # a pair at distance k+1 has a pair at distance k before it, so
            # no new pair now means none later
            break
        dist[hit] = k
        sigma[hit] = P[hit]
    return dist, sigma


def bc_brute(A: np.ndarray, S) -> np.ndarray:
    """BC[v] = sum over s in S, t != s, v != s, t of
    sigma_sv * sigma_vt / sigma_st whenever v lies on a shortest s-t path."""
    n = A.shape[0]
    dist, sigma = all_pairs_counts(A)
    bc = np.zeros(n, dtype=np.float64)
    for s in S:
        for t in range(n):
            if t == s or dist[s, t] < 0:
                continue
            for v in range(n):
                if v == s or v == t:
                    continue
                if dist[s, v] >= 0 and dist[v, t] >= 0 and dist[s, v] + dist[v, t] == dist[s, t]:
                    bc[v] += float(sigma[s, v] * sigma[v, t]) / float(sigma[s, t])
    return bc


def bc_sum_rhs(dist_rows: dict) -> int:
    """Right-hand side of the BC sum invariant: sum over sources s and
    reached targets t != s of (d(s,t) - 1)."""
    tot = 0
    for d in dist_rows.values():
        d = np.asarray(d, dtype=np.int64)
        r = d[d > 0]
        tot += int((r - 1).sum())
    return tot
