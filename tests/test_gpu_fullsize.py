"""Full-size parity: the workload shapes the benchmark and the batched /
betweenness configurations use, checked against the oracle on whole output
arrays where the oracle is fast enough, else on sampled sources plus the
BC sum invariant (sum_v BC[v] = sum_s sum_{t reached, t != s} (d(s,t) - 1),
right-hand side from oracle BFS distances)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from oracle import Oracle  # noqa: E402
from paper_2109_09527_amd import synth  # noqa: E402
from tests.pr_tolerance import assert_pr_close  # noqa: E402

BC_RTOL = 1e-9


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_09527_amd import dg as m
    return m


_T0 = [None]


def say(*a):
    import time
    if _T0[0] is None:
        _T0[0] = time.time()
    print("[case] %.1fs" % (time.time() - _T0[0]), *a, flush=True)


@pytest.mark.timeout(300)
def test_rmat20_update_batches_and_queries(dg):
    """R-MAT scale 20, 65,536 edge ops + 656 vertex ops per batch: every op
    result, and whole BFS / SSSP arrays after each batch."""
    wl = synth.update_batches(scale=20, n_batches=3, seed=0)
    gr = wl.graph
    say("rmat20 load", gr.m)
    o = Oracle(gr.n, w_max=255)
    g = dg.Graph(gr.n, w_max=255, edge_capacity=2 * gr.m)
    load = synth.load_ops(gr)
    rc, r_o = o.apply(load)
    res, _ = g.apply(dg.ops_to_device(load), torch.empty(len(load), dtype=torch.uint8, device="cuda"))
    for i, b in enumerate(wl.batches):
        say("rmat20 batch", i)
        rc, r_o = o.apply(b)
        res, ep = g.apply(b)
        assert np.array_equal(res, r_o)
        for s in (int(wl.bfs_src[i]), int(wl.sssp_src[i])):
            assert np.array_equal(g.bfs(s, ep).cpu().numpy(), o.bfs(s)[1])
            assert np.array_equal(g.sssp(s, ep).cpu().numpy(), o.sssp(s)[1])
    nv, na = g.stats()
    assert (nv, na) == o.counts()
    # snapshot PageRank of the last epoch, whole array (the per-vertex bound
    # of tests/pr_tolerance.py; iteration counts within one)
    say("rmat20 pagerank")
    rc, want, it_o, _ = o.pagerank()
    got, it, ch = g.pagerank(ep)
    r = assert_pr_close(got.cpu().numpy(), want, 1e-16, 0.85, o.counts()[0], "rmat20")
    say("rmat20 pagerank err/tol %.3g iterations %d vs %d" % (r, it, it_o))
    assert abs(it - it_o) <= 1 and ch <= 1e-16


@pytest.mark.timeout(600)
def test_rmat21_eight_epochs_batched_equals_plain(dg):
    """The batched configuration as stated: R-MAT scale 21 over 8 snapshot
    epochs (batches of log-uniform 64k-1M edge ops), 512 BFS/SSSP queries
    (50/50) in one engine call.  Every output equals the plain call element
    by element, and the oracle, replaying the batches in order, checks one
    BFS and one SSSP of every epoch on whole arrays (16 comparisons).  The
    configuration pairs query kind and epoch (query i is a BFS when i is
    even and binds epoch i mod 8), so each epoch's first batched query is
    compared, and the plain call of the other kind from the same source
    stands in for it (the batched and plain outputs are equal throughout)."""
    say("rmat21 generate")
    eq = synth.epoch_queries(scale=21, n_queries=512, seed=0)
    gr = eq.graph
    say("rmat21 load", gr.m)
    g = dg.Graph(gr.n, w_max=255, max_resident_epochs=8, edge_capacity=2 * gr.m)
    g.apply(dg.ops_to_device(synth.load_ops(gr)))
    epochs = [g.epoch]
    for b in eq.batches:
        _, ep = g.apply(dg.ops_to_device(b))
        epochs.append(ep)
        say("rmat21 epoch", ep, len(b))
    n = gr.n
    qs, outs = [], []
    for i in range(len(eq.kinds)):
        kind = dg.Q_BFS if eq.kinds[i] == 0 else dg.Q_SSSP
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        qs.append((kind, epochs[eq.epoch_slot[i]], int(eq.src[i]), out))
        outs.append(out)
    assert len(qs) == 512
    say("rmat21 batch of", len(qs))
    st = g.query_batch(qs)
    assert all(x == 0 for x in st)
    say("rmat21 plain comparison")
    for (kind, ep, s, out) in qs:
        plain = (g.bfs if kind == dg.Q_BFS else g.sssp)(s, ep)
        assert torch.equal(plain, out), (kind, ep, s)
    # the oracle at every epoch: its first batched query, and the plain
    # query of the other kind from the same source
    say("rmat21 oracle replay")
    o = Oracle(gr.n, w_max=255)
    o.apply(synth.load_ops(gr))
    checked = 0
    for k, ep in enumerate(epochs):
        if k > 0:
            o.apply(eq.batches[k - 1])
        assert o.epoch == ep
        kind, _, s, out = next(q for q in qs if q[1] == ep)
        other = (g.sssp if kind == dg.Q_BFS else g.bfs)(s, ep)
        for kk, got in ((kind, out), (dg.Q_SSSP if kind == dg.Q_BFS else dg.Q_BFS, other)):
            want = (o.bfs if kk == dg.Q_BFS else o.sssp)(s)[1]
            assert np.array_equal(got.cpu().numpy(), want), (kk, ep, s)
            checked += 1
        say("rmat21 oracle epoch", ep, "checked")
    assert checked == 16
    sample = [q for q in qs if q[1] == epochs[-1]][:1]
    # DFS collect at the last epoch: 2^21 vertices take the walk whose
    # discovered set is the disc array (the LDS bitmap would need 256 KB)
    s = sample[0][2]
    say("rmat21 dfs from", s)
    disc, par, nr = g.dfs(s, epochs[-1])
    _, wd, wp = o.dfs(s)
    assert np.array_equal(disc.cpu().numpy(), wd) and np.array_equal(par.cpu().numpy(), wp)
    assert nr == int((wd >= 0).sum())


@pytest.mark.timeout(600)
def test_rmat18_betweenness_before_and_after_deletions(dg):
    """Undirected unweighted R-MAT scale 18, 256 sources: BC within 1e-9 of
    the oracle on a source subset, the sum invariant over all 256 sources,
    the batched engine equal to the plain call; then again after 32,768
    undirected edge deletions."""
    wl = synth.bc_workload(scale=18, n_sources=256, seed=0)
    gr = wl.graph
    say("rmat18 load", gr.m)
    o = Oracle(gr.n, undirected=True, w_max=1)
    g = dg.Graph(gr.n, undirected=True, w_max=1, edge_capacity=4 * gr.m)
    o.apply(synth.load_ops(gr))
    g.apply(dg.ops_to_device(synth.load_ops(gr)))
    S = [int(x) for x in wl.sources]
    for phase in range(2):
        ep = g.epoch
        say("rmat18 bc phase", phase)
        bc_all = g.bc(S, ep).cpu().numpy()
        sub = S[:6]
        bc_sub = g.bc(sub, ep).cpu().numpy()
        want = o.bc(sub)[1]
        assert not (np.abs(bc_sub - want) > BC_RTOL * np.abs(want)).any()
        rhs = 0
        for s in S:
            d = o.bfs(s)[1].astype(np.int64)
            rhs += int((d[d > 0] - 1).sum())
        assert abs(bc_all.sum() - rhs) <= 1e-9 * rhs
        out = torch.empty(gr.n, dtype=torch.float64, device="cuda")
        st = g.query_batch([(dg.Q_BC, ep, sub, out)])
        assert st == [0] and np.array_equal(out.cpu().numpy(), bc_sub)
        if phase == 0:
            say("rmat18 deletions", len(wl.deletions))
            rc, r_o = o.apply(wl.deletions)
            res, _ = g.apply(wl.deletions)
            assert np.array_equal(res, r_o)
