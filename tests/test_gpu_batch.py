"""The persistent multi-query engine (dg_query_batch) against the plain
one-query calls and the oracle.

BFS / SSSP outputs must be bit-identical to the plain path and the oracle;
BC outputs bit-identical to the plain path (same per-vertex reduction
order) and within 1e-9 relative of the oracle.  Queries mix kinds and
epochs, include invalid ones, and run under several team sizes.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2109_09527_amd import synth  # noqa: E402

BC_RTOL = 1e-9


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_09527_amd import dg as m
    return m


def say(*a):
    print("[case]", *a, flush=True)


def build_history(dg, scale, undirected, n_batches, seed, w_max=60):
    gr = synth.rmat_graph(scale, 8, w_max, seed=seed, undirected=undirected,
                          unweighted=undirected)
    wmax = 1 if undirected else w_max
    o = Oracle(gr.n, undirected=undirected, w_max=wmax)
    g = dg.Graph(gr.n, undirected=undirected, w_max=wmax, max_resident_epochs=n_batches + 2)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    epochs = [g.epoch]
    if undirected:
        rng = np.random.default_rng(seed)
        batches = []
        for b in range(n_batches):
            pick = rng.choice(gr.m, size=min(500, gr.m), replace=False)
            batches.append(synth.make_ops(np.full(len(pick), synth.REME), gr.u[pick], gr.v[pick]))
    else:
        batches = synth.update_batches(graph=gr, n_batches=n_batches, n_edge_ops=1500, w_max=wmax,
                                       seed=seed).batches
    srcs = synth.out_degree_sources(gr, 6, synth.rng_for(seed, 5))
    answers = {}

    def record(ep):
        for s in srcs:
            s = int(s)
            answers[(ep, "bfs", s)] = o.bfs(s)
            answers[(ep, "sssp", s)] = o.sssp(s)
        S = [int(s) for s in srcs[:3] if o.alive(int(s))]
        answers[(ep, "bc", tuple(S))] = o.bc(S)

    record(g.epoch)
    for b in batches:
        o.apply(b)
        _, ep = g.apply(b)
        epochs.append(ep)
        record(ep)
    return gr, g, epochs, answers


def check_batch(dg, g, answers, shapes):
    """shapes: (workgroups per team, SSSP queries per lockstep launch)."""
    keys = list(answers.keys())
    n = g.n
    for S, G in shapes:
        g.set_tuning(batch_groups=S, batch_gang=G)
        say("batch team size", S, "gang", G, "queries", len(keys) + 3)
        queries, outs = [], []
        for (ep, kind, src) in keys:
            if kind == "bc":
                out = torch.empty(n, dtype=torch.float64, device="cuda")
                queries.append((dg.Q_BC, ep, list(src), out))
            else:
                out = torch.empty(n, dtype=torch.int32, device="cuda")
                queries.append((dg.Q_BFS if kind == "bfs" else dg.Q_SSSP, ep, src, out))
            outs.append(out)
        # invalid ones: unpublished epoch, out-of-range source, repeated BC source
        bad = [(dg.Q_BFS, g.epoch + 1, 0, torch.empty(n, dtype=torch.int32, device="cuda")),
               (dg.Q_SSSP, g.epoch, n + 5, torch.empty(n, dtype=torch.int32, device="cuda")),
               (dg.Q_BC, g.epoch, [keys[0][2], keys[0][2]], torch.empty(n, dtype=torch.float64, device="cuda"))]
        st = g.query_batch(queries + bad)
        torch.cuda.synchronize()
        assert st[-3] == dg.E_EPOCH_RETIRED
        assert st[-2] == dg.E_VERTEX_RANGE
        assert st[-1] == dg.E_INVALID_ARG
        for i, ((ep, kind, src), out) in enumerate(zip(keys, outs)):
            rc_o, want = answers[(ep, kind, src)]
            assert st[i] == rc_o, (kind, ep, src, st[i], rc_o)
            if rc_o != 0:
                continue
            got = out.cpu().numpy()
            if kind == "bc":
                plain = g.bc(list(src), ep).cpu().numpy()
                assert np.array_equal(got, plain), ("bc differs from plain", ep)
                err = np.abs(got - want)
                assert not (err > BC_RTOL * np.abs(want)).any(), ("bc vs oracle", ep)
            else:
                assert np.array_equal(got, want), (kind, ep, src, S)


@pytest.mark.parametrize("undirected", [False, True])
def test_batch_matches_plain_and_oracle(dg, undirected):
    gr, g, epochs, answers = build_history(dg, 11, undirected, 3, seed=7 + undirected)
    check_batch(dg, g, answers, [(0, 0), (1, 1), (3, 2), (16, 5)])
    with pytest.raises(dg.DGError):
        g.set_tuning(batch_gang=129)


def test_batch_many_queries_many_teams(dg):
    """Scale 13, 96 BFS/SSSP queries over 4 epochs, automatic teams."""
    gr = synth.rmat_graph(13, 16, 255, seed=11)
    o = Oracle(gr.n, w_max=255)
    g = dg.Graph(gr.n, w_max=255, max_resident_epochs=8)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    wl = synth.update_batches(graph=gr, n_batches=3, n_edge_ops=4000, seed=11)
    srcs = synth.out_degree_sources(gr, 24, synth.rng_for(11, 9))
    answers = {}
    for ep_i in range(4):
        ep = g.epoch
        for k, s in enumerate(srcs):
            s = int(s)
            if k % 2 == 0:
                answers[(ep, "bfs", s)] = o.bfs(s)
            else:
                answers[(ep, "sssp", s)] = o.sssp(s)
        if ep_i < 3:
            o.apply(wl.batches[ep_i])
            g.apply(wl.batches[ep_i])
    say("batch many queries")
    check_batch(dg, g, answers, [(0, 0), (2, 7)])


def test_autotune_keeps_results(dg):
    """The autotuner changes only speed: results after tuning equal the
    oracle's, and the chosen shape is one of the candidates."""
    gr = synth.rmat_graph(12, 16, 255, seed=21)
    o = Oracle(gr.n, w_max=255)
    g = dg.Graph(gr.n, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    say("autotune")
    t = g.autotune(seed=1)
    assert t["chunk_buckets"] in (16, 32, 64)
    assert t["sssp_delta"] in (16, 32, 64, 128, 256, 512)
    assert t["batch_delta"] in (64, 128, 256, 512, 1024, 2048)
    assert g.get_tuning() == t
    for s in synth.out_degree_sources(gr, 3, synth.rng_for(21, 2)):
        s = int(s)
        assert np.array_equal(g.bfs(s).cpu().numpy(), o.bfs(s)[1])
        assert np.array_equal(g.sssp(s).cpu().numpy(), o.sssp(s)[1])


@pytest.mark.parametrize("undirected", [False, True])
def test_multi_source_sssp_groups(dg, undirected):
    """SSSP queries of one snapshot run as multi-source searches of up to 16
    (one shared frontier, a vertex's distances for the group in one line).
    21 queries on the latest epoch (a group of 16, then one of 5) including
    a repeated source and a source without out-arcs, plus 6 on an earlier
    epoch read after a batch, at bucket widths from 1 to far above w_max:
    every output equals the oracle's Dijkstra."""
    gr = synth.rmat_graph(12, 16, 255, seed=23, undirected=undirected)
    o = Oracle(gr.n, undirected=undirected, w_max=255)
    g = dg.Graph(gr.n, undirected=undirected, w_max=255, max_resident_epochs=4)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    e0 = g.epoch
    srcs0 = [int(s) for s in synth.out_degree_sources(gr, 6, synth.rng_for(23, 4))]
    want0 = {s: o.sssp(s)[1] for s in srcs0}
    wl = synth.update_batches(graph=gr, n_batches=1, n_edge_ops=3000, w_max=255, seed=23)
    batch = wl.batches[0]
    batch = batch[(batch["type"] == synth.ADDE) | (batch["type"] == synth.REME)]   # every source stays live
    o.apply(batch)
    g.apply(batch)
    deg = np.bincount(np.concatenate([gr.u, gr.v]) if undirected else gr.u, minlength=gr.n)
    lone = [v for v in np.nonzero(deg == 0)[0][:50] if o.alive(int(v))][:1]
    srcs = [int(s) for s in synth.out_degree_sources(gr, 19, synth.rng_for(23, 5))]
    srcs = srcs[:10] + [srcs[0]] + [int(x) for x in lone] + srcs[10:]
    srcs = srcs[:21]
    want = {s: o.sssp(s)[1] for s in set(srcs)}
    for delta in (1, 7, 64, 255, 512, 100000):
        say("multi-source sssp delta", delta, "undirected", undirected)
        g.set_tuning(batch_delta=delta)
        q = [(dg.Q_SSSP, g.epoch, s, torch.empty(gr.n, dtype=torch.int32, device="cuda")) for s in srcs]
        q += [(dg.Q_SSSP, e0, s, torch.empty(gr.n, dtype=torch.int32, device="cuda")) for s in srcs0]
        st = g.query_batch(q)
        assert st == [0] * len(q)
        for i, (_, ep, s, out) in enumerate(q):
            ref = want[s] if ep != e0 else want0[s]
            assert np.array_equal(out.cpu().numpy(), ref), (delta, i, s, ep)


@pytest.mark.parametrize("undirected", [False, True])
def test_multi_source_bc_groups(dg, undirected):
    """BC queries of at least 4 sources run as multi-source searches of up
    to 16 sources (one shared frontier per level, a vertex's per-source
    state in one line per field).  Queries of 4, 16 and 21 sources (two
    groups) on the latest epoch and one of 7 on an earlier epoch read after
    a batch: every output equals the plain call bit for bit (same per-source
    summation order) and the oracle within 1e-9."""
    gr = synth.rmat_graph(11, 8, 1, seed=29, undirected=undirected, unweighted=True)
    o = Oracle(gr.n, undirected=undirected, w_max=1)
    g = dg.Graph(gr.n, undirected=undirected, w_max=1, max_resident_epochs=4)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    e0 = g.epoch
    S0 = [int(s) for s in synth.out_degree_sources(gr, 7, synth.rng_for(29, 4))]
    want0 = o.bc(S0)[1]
    rng = np.random.default_rng(29)
    pick = rng.choice(gr.m, size=gr.m // 10, replace=False)
    dels = synth.make_ops(np.full(len(pick), synth.REME), gr.u[pick], gr.v[pick])
    o.apply(dels)
    g.apply(dels)
    S = [int(s) for s in synth.out_degree_sources(gr, 21, synth.rng_for(29, 5))]
    cases = [(g.epoch, S[:4]), (g.epoch, S[:16]), (g.epoch, S), (e0, S0)]
    say("multi-source bc, undirected", undirected)
    outs = [torch.empty(gr.n, dtype=torch.float64, device="cuda") for _ in cases]
    st = g.query_batch([(dg.Q_BC, ep, srcs, out) for (ep, srcs), out in zip(cases, outs)])
    assert st == [0] * len(cases)
    for (ep, srcs), out in zip(cases, outs):
        got = out.cpu().numpy()
        plain = g.bc(srcs, ep).cpu().numpy()
        assert np.array_equal(got, plain), ("multi-source bc differs from plain", ep, len(srcs))
        want = want0 if ep == e0 else o.bc(srcs)[1]
        assert not (np.abs(got - want) > BC_RTOL * np.abs(want)).any(), ("bc vs oracle", ep, len(srcs))


def test_multi_source_bc_overflow(dg):
    """A chain of 63 diamonds has 2^63 shortest paths from its first vertex:
    a batched BC query of 4 sources that include it reports the overflow;
    one whose sources avoid it does not."""
    k = 63
    us, vs = [], []
    for i in range(k):
        a, b, c, d = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        us += [a, a, b, c]
        vs += [b, c, d, d]
    n = 3 * k + 1
    g = dg.Graph(n, w_max=1)
    g.apply(synth.make_ops([synth.ADDV] * n + [synth.ADDE] * len(us), list(range(n)) + us, [0] * n + vs,
                           [0] * n + [1] * len(us)))
    o1 = torch.empty(n, dtype=torch.float64, device="cuda")
    o2 = torch.empty(n, dtype=torch.float64, device="cuda")
    st = g.query_batch([(dg.Q_BC, g.epoch, [0, 3, 6, 9], o1), (dg.Q_BC, g.epoch, [3, 6, 9, 12], o2)])
    assert st[0] == dg.E_OVERFLOW
    assert st[1] == g.try_bc([3, 6, 9, 12])[0]


def test_multi_source_bfs_deep_levels(dg):
    """A directed path of 700 vertices plus a few shortcuts: a group of 6
    BFS queries reaches levels above 253, which no longer fit the group's
    one-byte level records and go to the outputs directly.  Every output
    equals the plain call and the oracle."""
    n = 700
    us = list(range(n - 1)) + [10, 300, 50]
    vs = list(range(1, n)) + [20, 320, 400]
    ops = synth.make_ops(np.array([synth.ADDV] * n + [synth.ADDE] * len(us), np.uint32),
                         np.array(list(range(n)) + us, np.uint32), np.array([0] * n + vs, np.uint32),
                         np.array([0] * n + [1] * len(us), np.int32))
    o = Oracle(n, w_max=1)
    g = dg.Graph(n, w_max=1)
    o.apply(ops)
    g.apply(ops)
    srcs = [0, 1, 2, 5, 30, 400]
    outs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in srcs]
    st = g.query_batch([(dg.Q_BFS, g.epoch, s, out) for s, out in zip(srcs, outs)])
    assert st == [0] * len(srcs)
    deepest = 0
    for s, out in zip(srcs, outs):
        got = out.cpu().numpy()
        want = o.bfs(s)[1]
        assert np.array_equal(got, want), s
        assert np.array_equal(got, g.bfs(s).cpu().numpy()), s
        deepest = max(deepest, int(got.max()))
    assert deepest > 300, deepest
