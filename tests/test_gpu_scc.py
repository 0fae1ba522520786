"""Parity of the snapshot traversals with the oracle: SCC labels (dg_scc,
smallest member, -1 for vertices not live) and component counts bit for bit;
the diameter (dg_diameter); the maximum flow value (dg_maxflow); and the DFS
preorder and tree parents (dg_dfs), which are unique for ascending neighbour
order, bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2109_09527_amd import synth  # noqa: E402
from paper_2109_09527_amd.synth import REME, REMV, make_ops  # noqa: E402


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_09527_amd import dg as m
    return m


def say(*a):
    print("[case]", *a, flush=True)


def build(dg, n, us, vs, undirected=False):
    us = np.asarray(us, dtype=np.uint32)
    vs = np.asarray(vs, dtype=np.uint32)
    gr = synth.Graph(n, us, vs, np.ones(len(us), np.int32), undirected)
    o = Oracle(n, undirected=undirected, w_max=255)
    g = dg.Graph(n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    return g, o


def check(g, o, epoch=None, want=None):
    if want is None:
        rc, want = o.scc()
        assert rc == 0
    comp, nc = g.scc(g.epoch if epoch is None else epoch)
    comp = comp.cpu().numpy()
    assert np.array_equal(comp, want), (np.nonzero(comp != want)[0][:10])
    assert nc == len(np.unique(want[want >= 0]))
    return comp


def test_closed_forms(dg):
    n = 30
    say("cycle")
    g, o = build(dg, n, np.arange(n), (np.arange(n) + 1) % n)
    assert np.all(check(g, o) == 0)
    say("path and reverse path")
    g, o = build(dg, n, np.arange(n - 1), np.arange(1, n))
    check(g, o)
    g, o = build(dg, n, np.arange(1, n), np.arange(n - 1))
    check(g, o)
    say("two cycles")
    g, o = build(dg, 7, [0, 1, 2, 3, 4, 5, 2], [1, 2, 0, 4, 5, 3, 3])
    assert check(g, o).tolist() == [0, 0, 0, 3, 3, 3, 6]
    say("undirected")
    g, o = build(dg, 6, [0, 3], [1, 4], undirected=True)
    assert check(g, o).tolist() == [0, 0, 2, 3, 3, 5]
    say("empty")
    g = dg.Graph(8, w_max=255)
    comp, nc = g.scc()
    assert nc == 0 and np.all(comp.cpu().numpy() == -1)


@pytest.mark.parametrize("undirected", [False, True])
def test_random_graphs_with_dead_vertices(dg, undirected):
    for seed in range(4):
        rng = synth.rng_for(seed, 93)
        n = 300
        m = 400 if undirected else 700
        us = rng.integers(0, n, m)
        vs = rng.integers(0, n, m)
        keep = us != vs
        say("random", undirected, seed)
        g, o = build(dg, n, us[keep], vs[keep], undirected)
        dead = rng.choice(n, 20, replace=False)
        ops = make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead)))
        o.apply(ops)
        g.apply(ops)
        check(g, o)


@pytest.mark.parametrize("undirected", [False, True])
def test_rmat_snapshots(dg, undirected):
    """R-MAT scale 14 (a giant component among many small ones, hubs with
    hundreds of buckets): the load epoch, pinned, and the epoch after edge
    removals, read afterwards."""
    gr = synth.rmat_graph(14, 8, 255, seed=23, undirected=undirected)
    o = Oracle(gr.n, undirected=undirected, w_max=255)
    g = dg.Graph(gr.n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    e1 = g.acquire()
    want1 = o.scc()[1]
    rng = synth.rng_for(23, 5)
    pick = rng.choice(gr.m, gr.m // 4, replace=False)
    ops = make_ops(np.full(len(pick), REME), gr.u[pick], gr.v[pick])
    o.apply(ops)
    g.apply(ops)
    say("rmat14 latest", undirected)
    check(g, o)
    say("rmat14 earlier", undirected)
    check(g, o, epoch=e1, want=want1)
    g.release(e1)


# ------------------------------------------------------------ diameter (GD)

def test_diameter_closed_forms(dg):
    n = 20
    say("diameter closed forms")
    cases = [
        ((np.arange(n - 1), np.arange(1, n)), False, n - 1),            # path
        ((np.arange(n), (np.arange(n) + 1) % n), False, n - 1),         # directed cycle
        ((np.arange(n), (np.arange(n) + 1) % n), True, n // 2),         # undirected cycle
        ((np.zeros(n - 1), np.arange(1, n)), False, 1),                 # out-star
        ((np.zeros(n - 1), np.arange(1, n)), True, 2),                  # undirected star
    ]
    for (us, vs), und, want in cases:
        g, o = build(dg, n, us, vs, und)
        assert g.diameter() == want == o.diameter()[1], (und, want)
    assert dg.Graph(8, w_max=255).diameter() == 0


@pytest.mark.parametrize("undirected", [False, True])
def test_diameter_random_and_rmat(dg, undirected):
    """Random graphs past one 256-source sweep, with dead vertices, and
    R-MAT 12 before and after edge removals (the earlier epoch read
    afterwards): equal to the oracle's BFS from every vertex."""
    for seed in range(3):
        rng = synth.rng_for(seed, 95)
        n = 700
        m = 900 if undirected else 1800
        us = rng.integers(0, n, m)
        vs = rng.integers(0, n, m)
        keep = us != vs
        say("diameter random", undirected, seed)
        g, o = build(dg, n, us[keep], vs[keep], undirected)
        dead = rng.choice(n, 30, replace=False)
        ops = make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead)))
        o.apply(ops)
        g.apply(ops)
        assert g.diameter() == o.diameter()[1]
    gr = synth.rmat_graph(12, 8, 255, seed=29, undirected=undirected)
    o = Oracle(gr.n, undirected=undirected, w_max=255)
    g = dg.Graph(gr.n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    e1 = g.acquire()
    want1 = o.diameter()[1]
    rng = synth.rng_for(29, 5)
    pick = rng.choice(gr.m, gr.m // 3, replace=False)
    ops = make_ops(np.full(len(pick), REME), gr.u[pick], gr.v[pick])
    o.apply(ops)
    g.apply(ops)
    say("diameter rmat12", undirected)
    assert g.diameter() == o.diameter()[1]
    assert g.diameter(e1) == want1
    g.release(e1)


# ------------------------------------------------------ network flow (GetNF)

def build_w(dg, n, us, vs, ws, undirected=False):
    gr = synth.Graph(n, np.asarray(us, np.uint32), np.asarray(vs, np.uint32), np.asarray(ws, np.int32), undirected)
    o = Oracle(n, undirected=undirected, w_max=255)
    g = dg.Graph(n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    return g, o


def test_maxflow_closed_forms_and_errors(dg):
    say("maxflow closed forms")
    g, o = build_w(dg, 4, [0, 1, 2], [1, 2, 3], [7, 3, 9])
    assert g.maxflow(0, 3) == 3 and g.maxflow(3, 0) == 0
    g, o = build_w(dg, 4, [0, 1, 0, 2], [1, 3, 2, 3], [5, 4, 6, 8])
    assert g.maxflow(0, 3) == 10
    # needs a reverse residual arc
    g, o = build_w(dg, 4, [0, 0, 1, 1, 2], [1, 2, 2, 3, 3], [1, 1, 1, 1, 1])
    assert g.maxflow(0, 3) == 2
    assert g.try_maxflow(1, 1)[0] == dg.E_INVALID_ARG
    assert g.try_maxflow(0, 99)[0] == dg.E_VERTEX_RANGE
    g.remove_vertex(2)
    assert g.try_maxflow(0, 2)[0] == dg.E_SOURCE_ABSENT


@pytest.mark.parametrize("undirected", [False, True])
def test_maxflow_random_and_rmat(dg, undirected):
    """Random weighted graphs and R-MAT 10 (weights 1..255), several
    source-sink pairs, before and after removals (the earlier epoch read
    afterwards): equal to the oracle's Edmonds-Karp."""
    for seed in range(3):
        rng = synth.rng_for(seed, 97)
        n = 60
        m = 150 if undirected else 300
        us = rng.integers(0, n, m)
        vs = rng.integers(0, n, m)
        keep = us != vs
        ws = rng.integers(1, 50, m)
        say("maxflow random", undirected, seed)
        g, o = build_w(dg, n, us[keep], vs[keep], ws[keep], undirected)
        for s, t in rng.integers(0, n, (6, 2)):
            if s != t:
                assert g.maxflow(int(s), int(t)) == o.maxflow(int(s), int(t))[1], (seed, s, t)
    gr = synth.rmat_graph(10, 8, 255, seed=31, undirected=undirected)
    o = Oracle(gr.n, undirected=undirected, w_max=255)
    g = dg.Graph(gr.n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    rng = synth.rng_for(31, 6)
    srcs = synth.out_degree_sources(gr, 6, rng)
    pairs = [(int(srcs[i]), int(srcs[i + 1])) for i in range(0, 6, 2)]
    e1 = g.acquire()
    want1 = [o.maxflow(s, t)[1] for s, t in pairs]
    pick = rng.choice(gr.m, gr.m // 4, replace=False)
    ops = make_ops(np.full(len(pick), REME), gr.u[pick], gr.v[pick])
    o.apply(ops)
    g.apply(ops)
    say("maxflow rmat10", undirected)
    for (s, t), w1 in zip(pairs, want1):
        assert g.maxflow(s, t) == o.maxflow(s, t)[1]
        assert g.maxflow(s, t, e1) == w1
    g.release(e1)


@pytest.mark.parametrize("undirected", [False, True])
def test_maxflow_rmat14(dg, undirected):
    """R-MAT scale 14 (weights 1..255 as capacities), four source-sink pairs
    with out-arcs, before and after removing an eighth of the edges (the
    earlier epoch read afterwards): flow values equal to the oracle's."""
    gr = synth.rmat_graph(14, 16, 255, seed=41, undirected=undirected)
    o = Oracle(gr.n, undirected=undirected, w_max=255)
    g = dg.Graph(gr.n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    rng = synth.rng_for(41, 6)
    srcs = synth.out_degree_sources(gr, 8, rng)
    pairs = [(int(srcs[i]), int(srcs[i + 1])) for i in range(0, 8, 2)]
    e1 = g.acquire()
    want1 = [o.maxflow(s, t)[1] for s, t in pairs]
    say("maxflow rmat14", undirected, want1)
    for (s, t), w1 in zip(pairs, want1):
        assert g.maxflow(s, t) == w1, (s, t)
    pick = rng.choice(gr.m, gr.m // 8, replace=False)
    ops = make_ops(np.full(len(pick), REME), gr.u[pick], gr.v[pick])
    o.apply(ops)
    g.apply(ops)
    say("maxflow rmat14 after removals", undirected)
    for (s, t), w1 in zip(pairs, want1):
        assert g.maxflow(s, t) == o.maxflow(s, t)[1], (s, t)
        assert g.maxflow(s, t, e1) == w1
    g.release(e1)


# ----------------------------------------------------- DFS collect (dg_dfs)

def dfs_equal(g, o, s, epoch=None, want=None):
    if want is None:
        rc, wd, wp = o.dfs(s)
        assert rc == 0
    else:
        wd, wp = want
    kw = {} if epoch is None else {"epoch": epoch}
    disc, par, nr = g.dfs(s, **kw)
    assert np.array_equal(disc.cpu().numpy(), wd), s
    assert np.array_equal(par.cpu().numpy(), wp), s
    assert nr == int((wd >= 0).sum())


def test_dfs_closed_forms_and_errors(dg):
    say("dfs closed forms")
    n = 300
    g, o = build(dg, n, np.arange(n - 1), np.arange(1, n))   # a path deeper than a wave
    disc, par, nr = g.dfs(0)
    assert np.array_equal(disc.cpu().numpy(), np.arange(n)) and nr == n
    dfs_equal(g, o, 150)
    # an out-star of 299 leaves, inserted in descending order (rows of several
    # 64-arc chunks)
    g, o = build(dg, n, np.zeros(n - 1), np.arange(n - 1, 0, -1))
    disc, par, nr = g.dfs(0)
    assert np.array_equal(disc.cpu().numpy(), np.arange(n))
    assert par.cpu().numpy().tolist() == [-1] + [0] * (n - 1)
    g, o = build(dg, 3, [0, 0, 1], [2, 1, 2])
    disc, par, _ = g.dfs(0)
    assert disc.cpu().tolist() == [0, 1, 2] and par.cpu().tolist() == [-1, 0, 1]
    # a hub whose row is scanned again, over several chunks, after a path
    # through its first neighbour has found every other one
    us = list(range(1, 200)) + [0] * 199
    vs = list(range(2, 201)) + list(range(1, 200))
    g, o = build(dg, 201, us, vs)
    dfs_equal(g, o, 0)
    assert g.try_dfs(10 ** 6)[0] == dg.E_VERTEX_RANGE
    g.remove_vertex(5)
    o.apply(make_ops(np.array([REMV]), np.array([5]), np.zeros(1)))
    assert g.try_dfs(5)[0] == dg.E_SOURCE_ABSENT
    dfs_equal(g, o, 0)


@pytest.mark.parametrize("undirected", [False, True])
def test_dfs_random_and_rmat(dg, undirected):
    """Random graphs with dead vertices and R-MAT 12 before and after removing
    a quarter of its edges (the earlier epoch read afterwards): preorder and
    parents equal to the oracle's for several sources."""
    for seed in range(3):
        rng = synth.rng_for(seed, 99)
        n = 500
        m = 900 if undirected else 1600
        us = rng.integers(0, n, m)
        vs = rng.integers(0, n, m)
        keep = us != vs
        say("dfs random", undirected, seed)
        g, o = build(dg, n, us[keep], vs[keep], undirected)
        dead = rng.choice(n, 10, replace=False)
        ops = make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead)))
        o.apply(ops)
        g.apply(ops)
        for s in rng.integers(0, n, 6).tolist():
            if o.alive(s):
                dfs_equal(g, o, s)
    gr = synth.rmat_graph(12, 16, 255, seed=41, undirected=undirected)
    g, o = build(dg, gr.n, gr.u, gr.v, undirected)
    rng = synth.rng_for(41, 3)
    srcs = [int(x) for x in synth.out_degree_sources(gr, 3, rng)]
    e1 = g.acquire()
    want1 = {s: o.dfs(s)[1:] for s in srcs}
    pick = rng.choice(gr.m, gr.m // 4, replace=False)
    ops = make_ops(np.full(len(pick), REME), gr.u[pick], gr.v[pick])
    o.apply(ops)
    g.apply(ops)
    say("dfs rmat12", undirected)
    for s in srcs:
        dfs_equal(g, o, s)
        dfs_equal(g, o, s, epoch=e1, want=want1[s])
    g.release(e1)


def test_dfs_abi_optional_outputs(dg):
    """dg_dfs through the C ABI with the optional parent array and reached
    count left null: disc alone, equal to the oracle's; a host disc array is
    rejected."""
    say("dfs abi optional outputs")
    rng = synth.rng_for(5, 99)
    n = 300
    us = rng.integers(0, n, 900)
    vs = rng.integers(0, n, 900)
    keep = us != vs
    g, o = build(dg, n, us[keep], vs[keep])
    disc = torch.empty(n, dtype=torch.int32, device="cuda")
    for s in (0, 17, 123):
        rc = dg.lib.dg_dfs(g.h, dg.EPOCH_LATEST, s, dg._ptr(disc), None, None, dg._stream())
        assert rc == 0
        assert np.array_equal(disc.cpu().numpy(), o.dfs(s)[1]), s
    host = np.zeros(n, dtype=np.int32)
    rc = dg.lib.dg_dfs(g.h, dg.EPOCH_LATEST, 0, host.ctypes.data, None, None, dg._stream())
    assert rc == dg.E_INVALID_ARG
