"""Seeded synthetic workloads for the dynamic-graph hot path.

This module only draws random inputs: graphs (Erdos-Renyi G(n, m) and R-MAT),
edge weights, operation batches and query sources.  It holds none of the
graph method's arithmetic (no batch resolution, no traversal); both the HIP
path and the CPU oracle consume exactly the arrays produced here.

Every generator takes an integer seed and derives independent sub-streams
from it with numpy's SeedSequence, so a workload is a pure function of
(config, seed).

Operation records use the 16-byte layout of the C boundary:
    u32 type, u32 u, u32 v, i32 w
with type codes AddVertex=0, RemoveVertex=1, ContainsVertex=2,
AddEdge=3, RemoveEdge=4, ContainsEdge=5 (the graph ADT operations
PutV/RemoveV/GetV/PutE/RemoveE/GetE named in the paper's preamble).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

OP_DTYPE = np.dtype([("type", "<u4"), ("u", "<u4"), ("v", "<u4"), ("w", "<i4")])
ADDV, REMV, HASV, ADDE, REME, HASE = range(6)

# Graph500-style R-MAT quadrant probabilities used by every R-MAT workload.
RMAT_ABC = (0.57, 0.19, 0.19)

# Sub-stream ids (one per kind of random draw).
_S_GRAPH, _S_WEIGHT, _S_OPS, _S_SRC, _S_ARRIVAL, _S_PERM = range(6)


def rng_for(seed: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream, sub])))


def make_ops(types, u, v, w=None) -> np.ndarray:
    n = len(types)
    ops = np.empty(n, dtype=OP_DTYPE)
    ops["type"] = types
    ops["u"] = u
    ops["v"] = v
    ops["w"] = 0 if w is None else w
    return ops


# ---------------------------------------------------------------- graphs

def er_edges(n: int, m: int, rng: np.random.Generator):
    """m distinct ordered pairs (u, v), u != v, uniform over all such pairs."""
    assert m <= n * (n - 1)
    keys = np.empty(0, dtype=np.int64)
    while len(keys) < m:
        k = max(2 * (m - len(keys)), 1024)
        u = rng.integers(0, n, k, dtype=np.int64)
        v = rng.integers(0, n, k, dtype=np.int64)
        ok = u != v
        cand = (u[ok] << 32) | v[ok]
        allk = np.concatenate([keys, cand])
        _, first = np.unique(allk, return_index=True)
        keys = allk[np.sort(first)]
    keys = keys[:m]
    return (keys >> 32).astype(np.uint32), (keys & 0xFFFFFFFF).astype(np.uint32)


def rmat_pairs(scale: int, k: int, rng: np.random.Generator, abc=RMAT_ABC):
    """k raw R-MAT samples (u, v) over [0, 2^scale), no noise, no relabelling."""
    a, b, c = abc
    u = np.zeros(k, dtype=np.uint32)
    v = np.zeros(k, dtype=np.uint32)
    t_ab, t_abc = a + b, a + b + c
    chunk = 1 << 22
    for lo in range(0, k, chunk):
        hi = min(k, lo + chunk)
        uu = np.zeros(hi - lo, dtype=np.uint32)
        vv = np.zeros(hi - lo, dtype=np.uint32)
        for _ in range(scale):
            r = rng.random(hi - lo, dtype=np.float32)
            ubit = r >= t_ab
            vbit = ((r >= a) & (r < t_ab)) | (r >= t_abc)
            uu = (uu << 1) | ubit.astype(np.uint32)
            vv = (vv << 1) | vbit.astype(np.uint32)
        u[lo:hi] = uu
        v[lo:hi] = vv
    return u, v


def dedup_pairs(u, v, undirected=False):
    """Drop self-loops and repeated keys; the first occurrence of a key wins.

    Returns the indices (into u, v) of the kept samples, in sample order.
    In undirected mode the key of (u, v) is {min, max}.
    """
    u64 = u.astype(np.int64)
    v64 = v.astype(np.int64)
    if undirected:
        a, b = np.minimum(u64, v64), np.maximum(u64, v64)
    else:
        a, b = u64, v64
    keep = np.nonzero(a != b)[0]
    keys = (a[keep] << 32) | b[keep]
    _, first = np.unique(keys, return_index=True)
    return keep[np.sort(first)]


@dataclass
class Graph:
    n: int
    u: np.ndarray           # uint32 endpoints, in load order
    v: np.ndarray
    w: np.ndarray           # int32 weights
    undirected: bool = False
    perm: np.ndarray | None = None   # R-MAT vertex relabelling (raw id -> id)

    @property
    def m(self) -> int:
        return len(self.u)


def rmat_graph(scale: int, edge_factor: int = 16, w_max: int = 255, seed: int = 0,
               undirected: bool = False, unweighted: bool = False) -> Graph:
    """R-MAT graph: edge_factor * 2^scale samples, seeded random relabelling,
    self-loops dropped, repeated keys dropped (first occurrence kept)."""
    n = 1 << scale
    g_rng = rng_for(seed, _S_GRAPH)
    u, v = rmat_pairs(scale, edge_factor * n, g_rng)
    perm = rng_for(seed, _S_PERM).permutation(n).astype(np.uint32)
    u, v = perm[u], perm[v]
    keep = dedup_pairs(u, v, undirected)
    u, v = u[keep], v[keep]
    if unweighted:
        w = np.ones(len(u), dtype=np.int32)
    else:
        w = rng_for(seed, _S_WEIGHT).integers(1, w_max + 1, len(u), dtype=np.int32)
    return Graph(n, u, v, w, undirected, perm)


def er_graph(n: int, m: int, w_max: int, seed: int = 0) -> Graph:
    u, v = er_edges(n, m, rng_for(seed, _S_GRAPH))
    w = rng_for(seed, _S_WEIGHT).integers(1, w_max + 1, m, dtype=np.int32)
    return Graph(n, u, v, w)


def load_ops(g: Graph) -> np.ndarray:
    """The initial bulk-load batch: AddVertex for every id in [0, n), then
    AddEdge for every edge of g in load order."""
    n, m = g.n, g.m
    types = np.concatenate([np.full(n, ADDV, np.uint32), np.full(m, ADDE, np.uint32)])
    uu = np.concatenate([np.arange(n, dtype=np.uint32), g.u])
    vv = np.concatenate([np.zeros(n, np.uint32), g.v])
    ww = np.concatenate([np.zeros(n, np.int32), g.w])
    return make_ops(types, uu, vv, ww)


def out_degree_sources(g: Graph, k: int, rng: np.random.Generator) -> np.ndarray:
    """k distinct vertices drawn uniformly among those with at least one
    out-arc in g (both endpoints count in undirected mode)."""
    if g.undirected:
        cand = np.unique(np.concatenate([g.u, g.v]))
    else:
        cand = np.unique(g.u)
    return rng.choice(cand, size=k, replace=False).astype(np.uint32)


# ---------------------------------------------------------- C1: tiny mixed

@dataclass
class Item:
    kind: str               # "batch" or "bfs" / "sssp" / "bc"
    ops: np.ndarray | None = None
    src: int = 0
    srcs: np.ndarray | None = None


def tiny_stream(n=1000, m=8000, n_ops=10_000, w_max=100, seed=0,
                mix=(0.2, 0.2, 0.1, 0.1, 0.2, 0.2)):
    """Erdos-Renyi graph plus a uniform mix of n_ops operations
    (AddEdge, RemoveEdge, AddVertex, RemoveVertex, ContainsEdge, BFS).

    Returns (graph, items): the load batch is items[0]; consecutive update
    ops between two queries form one batch; every BFS is a query item.
    AddEdge draws a uniform pair u != v; RemoveEdge / ContainsEdge target,
    with probability 1/2, an edge generated earlier (loaded or added), else a
    uniform pair.  Vertex ops and BFS sources draw from the ids the generator
    has itself added and not removed (its own bookkeeping of draws).
    """
    g = er_graph(n, m, w_max, seed)
    r = rng_for(seed, _S_OPS)
    pool = list(zip(g.u.tolist(), g.v.tolist()))
    live_ids = set(range(n))
    dead_ids = set()
    items = [Item("batch", load_ops(g))]
    cur = []
    kinds = r.choice(6, size=n_ops, p=np.asarray(mix))
    for k in kinds:
        if k == 0:      # AddEdge
            while True:
                u, v = int(r.integers(n)), int(r.integers(n))
                if u != v:
                    break
            cur.append((ADDE, u, v, int(r.integers(1, w_max + 1))))
            pool.append((u, v))
        elif k in (1, 4):   # RemoveEdge / ContainsEdge
            if r.random() < 0.5:
                u, v = pool[int(r.integers(len(pool)))]
            else:
                while True:
                    u, v = int(r.integers(n)), int(r.integers(n))
                    if u != v:
                        break
            cur.append((REME if k == 1 else HASE, u, v, 0))
        elif k == 2:    # AddVertex: prefer an id the generator removed
            if dead_ids and r.random() < 0.5:
                x = sorted(dead_ids)[int(r.integers(len(dead_ids)))]
            else:
                x = int(r.integers(n))
            dead_ids.discard(x)
            live_ids.add(x)
            cur.append((ADDV, x, 0, 0))
        elif k == 3:    # RemoveVertex of a (generator-side) live id
            x = sorted(live_ids)[int(r.integers(len(live_ids)))] if live_ids else int(r.integers(n))
            live_ids.discard(x)
            dead_ids.add(x)
            cur.append((REMV, x, 0, 0))
        else:           # BFS query from a generator-side live id
            if cur:
                a = np.array(cur, dtype=np.int64)
                items.append(Item("batch", make_ops(a[:, 0], a[:, 1], a[:, 2], a[:, 3])))
                cur = []
            s = sorted(live_ids)[int(r.integers(len(live_ids)))] if live_ids else 0
            items.append(Item("bfs", src=s))
    if cur:
        a = np.array(cur, dtype=np.int64)
        items.append(Item("batch", make_ops(a[:, 0], a[:, 1], a[:, 2], a[:, 3])))
    return g, items


# ------------------------------------------------- C2: R-MAT update batches

@dataclass
class BatchWorkload:
    graph: Graph
    batches: list = field(default_factory=list)     # list of op arrays
    bfs_src: np.ndarray | None = None               # one source per batch
    sssp_src: np.ndarray | None = None
    w_max: int = 255


def update_batches(scale=20, n_batches=64, n_edge_ops=65_536, vertex_frac=0.01,
                   w_max=255, seed=0, edge_factor=16, graph: Graph | None = None):
    """R-MAT graph plus n_batches batches of n_edge_ops edge ops (half AddEdge
    with fresh R-MAT endpoints, half RemoveEdge drawn without replacement, per
    batch, from the edges generated so far) and vertex_frac * n_edge_ops vertex
    ops (half AddVertex on a uniform id, half RemoveVertex on a uniform id
    that is not a query source), shuffled.  One BFS and one SSSP source per
    batch are drawn up front among vertices with an initial out-arc; they are
    never the target of a RemoveVertex.
    """
    g = graph if graph is not None else rmat_graph(scale, edge_factor, w_max, seed)
    n = g.n
    r = rng_for(seed, _S_OPS)
    src = out_degree_sources(g, 2 * n_batches, rng_for(seed, _S_SRC))
    protected = np.zeros(n, dtype=bool)
    protected[src] = True
    pool_u, pool_v = [g.u], [g.v]
    pool_len = g.m
    n_add = n_edge_ops // 2
    n_rem = n_edge_ops - n_add
    n_vx = int(round(vertex_frac * n_edge_ops))
    n_addv = n_vx // 2
    n_remv = n_vx - n_addv
    scale_bits = int(math.log2(n))
    perm = g.perm
    batches = []
    for _ in range(n_batches):
        # fresh R-MAT endpoints for AddEdge (self-loops redrawn)
        au = np.empty(0, np.uint32)
        av = np.empty(0, np.uint32)
        while len(au) < n_add:
            uu, vv = rmat_pairs(scale_bits, 2 * (n_add - len(au)) + 64, r)
            if perm is not None:
                uu, vv = perm[uu], perm[vv]
            ok = uu != vv
            au = np.concatenate([au, uu[ok]])
            av = np.concatenate([av, vv[ok]])
        au, av = au[:n_add], av[:n_add]
        aw = r.integers(1, w_max + 1, n_add, dtype=np.int32)
        pu = np.concatenate(pool_u) if len(pool_u) > 1 else pool_u[0]
        pv = np.concatenate(pool_v) if len(pool_v) > 1 else pool_v[0]
        pool_u, pool_v = [pu], [pv]
        pick = r.choice(pool_len, size=n_rem, replace=False)
        ru, rv = pu[pick], pv[pick]
        addv = r.integers(0, n, n_addv, dtype=np.uint32)
        remv = np.empty(0, np.uint32)
        while len(remv) < n_remv:
            c = r.integers(0, n, 2 * n_remv + 8, dtype=np.uint32)
            remv = np.concatenate([remv, c[~protected[c]]])
        remv = remv[:n_remv]
        types = np.concatenate([np.full(n_add, ADDE, np.uint32), np.full(n_rem, REME, np.uint32),
                                np.full(n_addv, ADDV, np.uint32), np.full(n_remv, REMV, np.uint32)])
        uu = np.concatenate([au, ru, addv, remv])
        vv = np.concatenate([av, rv, np.zeros(n_vx, np.uint32)])
        ww = np.concatenate([aw, np.zeros(n_rem + n_vx, np.int32)])
        order = r.permutation(len(types))
        batches.append(make_ops(types[order], uu[order], vv[order], ww[order]))
        pool_u.append(au)
        pool_v.append(av)
        pool_len += n_add
    return BatchWorkload(g, batches, src[:n_batches], src[n_batches:], w_max)


# ------------------------------------------- C3: queries over several epochs

@dataclass
class EpochQueries:
    graph: Graph
    batches: list                 # one edge-op batch per extra epoch
    kinds: np.ndarray             # 0 = BFS, 1 = SSSP, per query
    epoch_slot: np.ndarray        # 0 = after the load, k = after batches[k-1]
    src: np.ndarray


def epoch_queries(scale=21, n_epochs=8, n_queries=512, min_ops=65_536, max_ops=1_048_576,
                  w_max=255, seed=0, edge_factor=16, graph: Graph | None = None):
    """R-MAT graph loaded as the first snapshot, then n_epochs - 1 batches of
    log-uniform[min_ops, max_ops] edge ops (half AddEdge with R-MAT endpoints,
    half RemoveEdge drawn from the generated edges), one snapshot per batch.
    Query i is a BFS when i is even, an SSSP when odd, on snapshot i mod
    n_epochs, from a source with an initial out-arc (no vertex ops here, so
    every source stays live)."""
    g = graph if graph is not None else rmat_graph(scale, edge_factor, w_max, seed)
    r = rng_for(seed, _S_OPS)
    scale_bits = int(math.log2(g.n))
    pu, pv = g.u, g.v
    batches = []
    for _ in range(n_epochs - 1):
        k = int(math.exp(r.uniform(math.log(min_ops), math.log(max_ops))))
        n_add = k // 2
        n_rem = k - n_add
        uu, vv = rmat_pairs(scale_bits, n_add + n_add // 8 + 64, r)
        uu, vv = g.perm[uu], g.perm[vv]
        ok = uu != vv
        au, av = uu[ok][:n_add], vv[ok][:n_add]
        aw = r.integers(1, w_max + 1, len(au), dtype=np.int32)
        pick = r.choice(len(pu), size=n_rem, replace=False)
        types = np.concatenate([np.full(len(au), ADDE, np.uint32), np.full(n_rem, REME, np.uint32)])
        ou = np.concatenate([au, pu[pick]])
        ov = np.concatenate([av, pv[pick]])
        ow = np.concatenate([aw, np.zeros(n_rem, np.int32)])
        order = r.permutation(len(types))
        batches.append(make_ops(types[order], ou[order], ov[order], ow[order]))
        pu = np.concatenate([pu, au])
        pv = np.concatenate([pv, av])
    src = rng_for(seed, _S_SRC).choice(np.unique(g.u), size=n_queries, replace=True).astype(np.uint32)
    kinds = (np.arange(n_queries) % 2).astype(np.uint32)
    slot = (np.arange(n_queries) % n_epochs).astype(np.uint32)
    return EpochQueries(g, batches, kinds, slot, src)


# ------------------------------------------------- C4: betweenness workload

@dataclass
class BCWorkload:
    graph: Graph
    sources: np.ndarray
    deletions: np.ndarray         # RemoveEdge batch applied between the two runs


def bc_workload(scale=18, n_sources=256, n_deletions=32_768, seed=0, edge_factor=16):
    """Undirected unweighted R-MAT graph, n_sources distinct sources among
    non-isolated vertices, and a batch of n_deletions undirected RemoveEdge
    ops drawn without replacement from the loaded edges."""
    g = rmat_graph(scale, edge_factor, 1, seed, undirected=True, unweighted=True)
    S = out_degree_sources(g, n_sources, rng_for(seed, _S_SRC))
    pick = rng_for(seed, _S_OPS).choice(g.m, size=min(n_deletions, g.m), replace=False)
    dels = make_ops(np.full(len(pick), REME, np.uint32), g.u[pick], g.v[pick])
    return BCWorkload(g, S, dels)


# ------------------------------------------------------ C5: serving arrivals

@dataclass
class Request:
    t: float                      # arrival time, seconds from start
    kind: str                     # "update", "bfs", "sssp", "bc"
    ops: np.ndarray | None = None
    src: int = 0
    srcs: np.ndarray | None = None


def serving_requests(g: Graph, rate=2000.0, duration=1.0, seed=0, w_max=255,
                     min_upd=1024, max_upd=262_144, bc_sources=16,
                     mix=(0.3, 0.28, 0.28, 0.14)):
    """Open-loop Poisson arrivals at `rate` per second for `duration` seconds.
    Mix (update, BFS, SSSP, BC): 30% update batches of log-uniform
    [min_upd, max_upd] edge ops (half AddEdge with R-MAT endpoints, half
    RemoveEdge of generated edges); 70% queries split 40/40/20 between BFS,
    SSSP and BC with bc_sources sources."""
    r = rng_for(seed, _S_ARRIVAL)
    ro = rng_for(seed, _S_OPS)
    rs = rng_for(seed, _S_SRC)
    scale_bits = int(math.log2(g.n))
    cand = np.unique(g.u)
    t = 0.0
    reqs = []
    pu, pv = g.u, g.v
    while True:
        t += float(r.exponential(1.0 / rate))
        if t >= duration:
            break
        k = int(r.choice(4, p=np.asarray(mix)))
        if k == 0:
            nops = int(math.exp(ro.uniform(math.log(min_upd), math.log(max_upd))))
            n_add = nops // 2
            n_rem = nops - n_add
            uu, vv = rmat_pairs(scale_bits, n_add + n_add // 8 + 64, ro)
            uu, vv = g.perm[uu], g.perm[vv]
            ok = uu != vv
            au, av = uu[ok][:n_add], vv[ok][:n_add]
            aw = ro.integers(1, w_max + 1, len(au), dtype=np.int32)
            pick = ro.integers(0, len(pu), n_rem)
            types = np.concatenate([np.full(len(au), ADDE, np.uint32), np.full(n_rem, REME, np.uint32)])
            ops = make_ops(types, np.concatenate([au, pu[pick]]), np.concatenate([av, pv[pick]]),
                           np.concatenate([aw, np.zeros(n_rem, np.int32)]))
            ops = ops[ro.permutation(len(ops))]
            reqs.append(Request(t, "update", ops=ops))
        elif k == 1:
            reqs.append(Request(t, "bfs", src=int(rs.choice(cand))))
        elif k == 2:
            reqs.append(Request(t, "sssp", src=int(rs.choice(cand))))
        else:
            reqs.append(Request(t, "bc", srcs=rs.choice(cand, size=bc_sources, replace=False).astype(np.uint32)))
    return reqs


# ------------------------------------------------------ small test graphs

def random_small_graph(n: int, p: float, seed: int, w_max: int = 9, undirected=False):
    """Dense-ish random graph for brute-force checks: each ordered pair
    (unordered in undirected mode) is an edge with probability p."""
    r = rng_for(seed, _S_GRAPH, 7)
    us, vs = np.nonzero(r.random((n, n)) < p)
    ok = us != vs
    us, vs = us[ok], vs[ok]
    if undirected:
        ok = us < vs
        us, vs = us[ok], vs[ok]
    w = r.integers(1, w_max + 1, len(us), dtype=np.int32)
    return Graph(n, us.astype(np.uint32), vs.astype(np.uint32), w, undirected)


def random_ops(n: int, k: int, seed: int, w_max: int = 9, mix=None):
    """k uniformly mixed ops over ids [0, n) (all six types)."""
    r = rng_for(seed, _S_OPS, 11)
    types = r.choice(6, size=k, p=mix).astype(np.uint32)
    u = r.integers(0, n, k, dtype=np.uint32)
    v = r.integers(0, n, k, dtype=np.uint32)
    w = r.integers(1, w_max + 1, k, dtype=np.int32)
    return make_ops(types, u, v, w)
