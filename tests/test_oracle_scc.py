"""Pins for the oracle's strongly connected components (CPU only).

Definition: u and v share a component iff each reaches the other (or
u = v); the label is the smallest id in the component, -1 for vertices that
are not live.  Checked against that definition through Warshall's closure
on random graphs with dead vertices, against closed forms, and on a larger
R-MAT graph against invariants: labels are fixed points at or below their
vertex, and the condensation has no cycle.
"""
import numpy as np
import pytest

from oracle import Oracle, OK, E_INVALID_ARG
from paper_2109_09527_amd import synth
from paper_2109_09527_amd.synth import REMV, make_ops
from tests.brute import warshall


def load(n, us, vs, undirected=False):
    o = Oracle(n, undirected=undirected, w_max=255)
    us = np.asarray(us, dtype=np.uint32)
    vs = np.asarray(vs, dtype=np.uint32)
    g = synth.Graph(n, us, vs, np.ones(len(us), np.int32), undirected)
    rc, _ = o.apply(synth.load_ops(g))
    assert rc == OK
    return o


def brute_labels(o):
    n = o.n
    live = np.array([o.alive(v) for v in range(n)])
    A = np.zeros((n, n), dtype=bool)
    us, vs, _ = o.edges()
    A[us, vs] = True
    if o.undirected:
        A[vs, us] = True
    R = warshall(A) | np.eye(n, dtype=bool)
    same = R & R.T
    lab = np.full(n, -1, dtype=np.int32)
    for v in range(n):
        if live[v]:
            lab[v] = int(np.nonzero(same[v] & live)[0].min())
    return lab


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_matches_reachability_definition(seed, undirected):
    rng = synth.rng_for(seed, 92)
    n = 40
    m = 60 if undirected else 90
    us = rng.integers(0, n, m)
    vs = rng.integers(0, n, m)
    keep = us != vs
    o = load(n, us[keep], vs[keep], undirected)
    dead = rng.choice(n, 4, replace=False)
    o.apply(make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead))))
    rc, lab = o.scc()
    assert rc == OK
    assert np.array_equal(lab, brute_labels(o))


def test_closed_forms():
    n = 30
    cyc = load(n, np.arange(n), (np.arange(n) + 1) % n)
    assert np.all(cyc.scc()[1] == 0)
    path = load(n, np.arange(n - 1), np.arange(1, n))
    assert np.array_equal(path.scc()[1], np.arange(n))
    # two 3-cycles {0,1,2} and {3,4,5} joined by 2 -> 3, and an isolated 6
    two = load(7, [0, 1, 2, 3, 4, 5, 2], [1, 2, 0, 4, 5, 3, 3])
    assert two.scc()[1].tolist() == [0, 0, 0, 3, 3, 3, 6]
    # a reverse path has its largest id first: still singletons
    rev = load(n, np.arange(1, n), np.arange(n - 1))
    assert np.array_equal(rev.scc()[1], np.arange(n))
    # undirected: connected components
    und = load(6, [0, 3], [1, 4], undirected=True)
    assert und.scc()[1].tolist() == [0, 0, 2, 3, 3, 5]


def test_rmat_invariants():
    gr = synth.rmat_graph(12, 8, 255, seed=6)
    o = load(gr.n, gr.u, gr.v)
    rc, lab = o.scc()
    assert rc == OK
    assert np.all(lab <= np.arange(gr.n)) and np.array_equal(lab[lab], lab)
    # condensation: order the components so every cross arc goes forward
    us, vs, _ = o.edges()
    a, b = lab[us], lab[vs]
    cross = a != b
    comps = np.unique(lab)
    idx = {c: i for i, c in enumerate(comps.tolist())}
    indeg = np.zeros(len(comps), dtype=np.int64)
    adj = [[] for _ in comps]
    for x, y in set(zip(a[cross].tolist(), b[cross].tolist())):
        adj[idx[x]].append(idx[y])
        indeg[idx[y]] += 1
    queue = [i for i in range(len(comps)) if indeg[i] == 0]
    seen = 0
    while queue:
        i = queue.pop()
        seen += 1
        for j in adj[i]:
            indeg[j] -= 1
            if indeg[j] == 0:
                queue.append(j)
    assert seen == len(comps)   # acyclic
    # the graph has one large component besides many singletons
    sizes = np.bincount(lab)
    assert sizes.max() > gr.n // 4


# ------------------------------------------------------------ diameter (GD)

def brute_diameter(o):
    """Largest finite hop distance from Floyd-Warshall on the arc matrix."""
    n = o.n
    live = np.array([o.alive(v) for v in range(n)])
    INF = 10 ** 9
    D = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(D, 0)
    us, vs, _ = o.edges()
    D[us, vs] = np.minimum(D[us, vs], 1)
    if o.undirected:
        D[vs, us] = np.minimum(D[vs, us], 1)
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    D = D[np.ix_(live, live)]
    fin = D[D < INF]
    return int(fin.max()) if fin.size else 0


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_diameter_matches_floyd_warshall(seed, undirected):
    rng = synth.rng_for(seed, 94)
    n = 40
    m = 50 if undirected else 80
    us = rng.integers(0, n, m)
    vs = rng.integers(0, n, m)
    keep = us != vs
    o = load(n, us[keep], vs[keep], undirected)
    dead = rng.choice(n, 3, replace=False)
    o.apply(make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead))))
    rc, d = o.diameter()
    assert rc == OK and d == brute_diameter(o)


def test_diameter_closed_forms():
    n = 20
    assert load(n, np.arange(n - 1), np.arange(1, n)).diameter()[1] == n - 1          # path
    assert load(n, np.arange(n), (np.arange(n) + 1) % n).diameter()[1] == n - 1       # directed cycle
    assert load(n, np.arange(n), (np.arange(n) + 1) % n, undirected=True).diameter()[1] == n // 2
    assert load(n, np.zeros(n - 1), np.arange(1, n)).diameter()[1] == 1               # out-star
    assert load(n, np.zeros(n - 1), np.arange(1, n), undirected=True).diameter()[1] == 2
    assert Oracle(5).diameter()[1] == 0


# ------------------------------------------------------ network flow (GetNF)

def load_w(n, us, vs, ws, undirected=False):
    o = Oracle(n, undirected=undirected, w_max=255)
    g = synth.Graph(n, np.asarray(us, np.uint32), np.asarray(vs, np.uint32), np.asarray(ws, np.int32), undirected)
    rc, _ = o.apply(synth.load_ops(g))
    assert rc == OK
    return o


def brute_min_cut(o, s, t):
    """Max-flow min-cut: the least total weight of arcs leaving a vertex set
    that holds s and not t, over all such sets."""
    n = o.n
    us, vs, ws = o.edges()
    arcs = list(zip(us.tolist(), vs.tolist(), ws.tolist()))
    if o.undirected:
        arcs += [(b, a, w) for a, b, w in arcs if a != b]
    others = [v for v in range(n) if v not in (s, t)]
    best = None
    for mask in range(1 << len(others)):
        S = {s} | {others[i] for i in range(len(others)) if mask >> i & 1}
        cut = sum(w for a, b, w in arcs if a in S and b not in S)
        best = cut if best is None else min(best, cut)
    return best


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_maxflow_equals_min_cut(seed, undirected):
    rng = synth.rng_for(seed, 96)
    n = 11
    m = 20 if undirected else 35
    us = rng.integers(0, n, m)
    vs = rng.integers(0, n, m)
    keep = us != vs
    ws = rng.integers(1, 20, m)
    o = load_w(n, us[keep], vs[keep], ws[keep], undirected)
    for s, t in ((0, n - 1), (3, 5), (n - 1, 0)):
        rc, f = o.maxflow(s, t)
        assert rc == OK and f == brute_min_cut(o, s, t), (s, t)


def test_maxflow_closed_forms():
    # a path: its lightest arc; two disjoint paths: the sum; no path: 0
    path = load_w(4, [0, 1, 2], [1, 2, 3], [7, 3, 9])
    assert path.maxflow(0, 3) == (OK, 3)
    assert path.maxflow(3, 0) == (OK, 0)
    two = load_w(4, [0, 1, 0, 2], [1, 3, 2, 3], [5, 4, 6, 8])
    assert two.maxflow(0, 3) == (OK, 10)
    # a flow that must use a reverse residual arc (the classic crossing)
    x = load_w(4, [0, 0, 1, 1, 2], [1, 2, 2, 3, 3], [1, 1, 1, 1, 1])
    assert x.maxflow(0, 3) == (OK, 2)
    assert path.maxflow(1, 1)[0] == E_INVALID_ARG


# ----------------------------------------------------- DFS collect (GetDFS)

def recursive_dfs(o, s):
    """Textbook recursive DFS, neighbours in ascending id order."""
    import sys
    n = o.n
    us, vs, _ = o.edges()
    adj = [[] for _ in range(n)]
    for a, b in zip(us.tolist(), vs.tolist()):
        adj[a].append(b)
        if o.undirected and a != b:
            adj[b].append(a)
    disc = [-1] * n
    par = [-1] * n
    clock = [0]

    def visit(x):
        disc[x] = clock[0]
        clock[0] += 1
        for y in sorted(adj[x]):
            if disc[y] < 0:
                par[y] = x
                visit(y)

    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 4 * n + 100))
    try:
        visit(s)
    finally:
        sys.setrecursionlimit(old)
    return np.array(disc, np.int32), np.array(par, np.int32)


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_dfs_matches_recursive_definition(seed, undirected):
    rng = synth.rng_for(seed, 98)
    n = 40
    m = 60 if undirected else 100
    us = rng.integers(0, n, m)
    vs = rng.integers(0, n, m)
    keep = us != vs
    o = load(n, us[keep], vs[keep], undirected)
    dead = rng.choice(n, 3, replace=False)
    o.apply(make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead))))
    for s in range(n):
        if not o.alive(s):
            continue
        rc, disc, par = o.dfs(s)
        assert rc == OK
        want_d, want_p = recursive_dfs(o, s)
        assert np.array_equal(disc, want_d) and np.array_equal(par, want_p), s


def test_dfs_closed_forms():
    n = 12
    path = load(n, np.arange(n - 1), np.arange(1, n))
    rc, disc, par = path.dfs(0)
    assert rc == OK and np.array_equal(disc, np.arange(n)) and par.tolist() == [-1] + list(range(n - 1))
    # preorder, not postorder: from the middle only the tail is reached
    rc, disc, par = path.dfs(5)
    assert disc.tolist() == [-1] * 5 + list(range(n - 5))
    # an out-star inserted in descending order is still visited ascending
    star = load(n, np.zeros(n - 1), np.arange(n - 1, 0, -1))
    rc, disc, par = star.dfs(0)
    assert np.array_equal(disc, np.arange(n)) and par.tolist() == [-1] + [0] * (n - 1)
    # 0 -> 2, 0 -> 1, 1 -> 2: 2 is found through 1
    tri = load(3, [0, 0, 1], [2, 1, 2])
    assert [a.tolist() for a in tri.dfs(0)[1:]] == [[0, 1, 2], [-1, 0, 1]]
    # a reverse path from its top
    rev = load(n, np.arange(1, n), np.arange(n - 1))
    rc, disc, par = rev.dfs(n - 1)
    assert np.array_equal(disc, np.arange(n - 1, -1, -1))
    assert path.dfs(n + 3)[0] != OK
    path.apply(make_ops(np.array([REMV]), np.array([3]), np.zeros(1)))
    assert path.dfs(3)[0] != OK


@pytest.mark.parametrize("undirected", [False, True])
def test_dfs_rmat_invariants(undirected):
    """Properties that fix a DFS in ascending neighbour order: the reached set
    is BFS's; the tree arcs are arcs; every arc from an earlier-discovered
    vertex leads into its subtree (white-path theorem); and a parent's
    smaller neighbours were all discovered before its child."""
    gr = synth.rmat_graph(11, 8, 255, seed=8, undirected=undirected)
    o = load(gr.n, gr.u, gr.v, undirected)
    s = int(synth.out_degree_sources(gr, 1, synth.rng_for(8, 1))[0])
    rc, disc, par = o.dfs(s)
    assert rc == OK
    reached = disc >= 0
    assert np.array_equal(reached, o.bfs(s)[1] >= 0)
    r = int(reached.sum())
    assert sorted(disc[reached].tolist()) == list(range(r))
    us, vs, _ = o.edges()
    if undirected:
        us, vs = np.concatenate([us, vs]), np.concatenate([vs, us])
    arcs = set(zip(us.tolist(), vs.tolist()))
    kids = [[] for _ in range(o.n)]
    for v in np.nonzero(reached)[0].tolist():
        p = int(par[v])
        if v == s:
            assert p == -1
            continue
        assert (p, v) in arcs and disc[p] < disc[v]
        kids[p].append(v)
    size = np.zeros(o.n, np.int64)
    for v in sorted(np.nonzero(reached)[0].tolist(), key=lambda x: -disc[x]):
        size[v] = 1 + sum(size[c] for c in kids[v])
    nbrs = [[] for _ in range(o.n)]
    for a, b in arcs:
        nbrs[a].append(b)
    for a, b in arcs:
        if reached[a]:
            assert reached[b]
            if disc[a] < disc[b]:
                assert disc[b] < disc[a] + size[a], (a, b)
    for v in np.nonzero(reached)[0].tolist():
        if v != s:
            p = int(par[v])
            assert all(disc[y] < disc[v] for y in nbrs[p] if y < v), v
