"""Parity of the plain HIP path (one query per call) with the CPU oracle.

Op results, BFS and SSSP distances must be bit-exact; BC within 1e-9
relative per vertex (exact 0 where the oracle has 0), as the path computes
int64 path counts and FP64 dependencies in a different summation order.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2109_09527_amd import synth  # noqa: E402
from paper_2109_09527_amd.synth import ADDV, REMV, HASV, ADDE, REME, HASE, make_ops  # noqa: E402

BC_RTOL = 1e-9


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_09527_amd import dg as m
    return m


def say(*a):
    print("[case]", *a, flush=True)


def assert_bc_close(got, want):
    got = np.asarray(got)
    want = np.asarray(want)
    err = np.abs(got - want)
    bad = err > BC_RTOL * np.abs(want)
    assert not bad.any(), (np.nonzero(bad)[0][:10], got[bad][:10], want[bad][:10])


def check_queries(g, o, e, srcs, dg, bc=False):
    for s in srcs:
        s = int(s)
        rc_o, d_o = o.bfs(s)
        rc, d = g.try_bfs(s, e)
        assert rc == rc_o, ("bfs status", s, rc, rc_o)
        if rc == 0:
            assert np.array_equal(d.cpu().numpy(), d_o), ("bfs", s)
        rc_o, d_o = o.sssp(s)
        rc, d = g.try_sssp(s, e)
        assert rc == rc_o, ("sssp status", s, rc, rc_o)
        if rc == 0:
            assert np.array_equal(d.cpu().numpy(), d_o), ("sssp", s)
    if bc:
        S = [int(s) for s in srcs if o.alive(int(s))]
        if S:
            rc_o, b_o = o.bc(S)
            rc, b = g.try_bc(S, e)
            assert rc == rc_o
            if rc == 0:
                assert_bc_close(b.cpu().numpy(), b_o)


def test_golden_scenario_on_gpu(dg):
    from tests.golden_io import read_adt_scenario
    n, steps = read_adt_scenario("adt_directed.txt")
    g = dg.Graph(n, w_max=9)
    say("golden scenario")
    for st in steps:
        if st[0] == "op":
            res, _ = g.apply(st[1])
            assert int(res[0]) == st[2], st
        else:
            kind, s, want = st[1], st[2], st[3]
            d = g.bfs(s) if kind == "bfs" else g.sssp(s)
            assert np.array_equal(d.cpu().numpy(), want), (kind, s)


def test_tiny_er_workload_full_parity(dg):
    """ER 1,000 / 8,000, 10,000 mixed ops: every op result and every BFS."""
    gr, items = synth.tiny_stream()
    o = Oracle(gr.n, w_max=100)
    g = dg.Graph(gr.n, w_max=100, edge_capacity=16000)
    say("tiny ER workload")
    nb = nq = 0
    for it in items:
        if it.kind == "batch":
            rc_o, r_o = o.apply(it.ops)
            res, ep = g.apply(it.ops)
            assert np.array_equal(res, r_o), ("batch", nb, np.nonzero(res != r_o)[0][:10])
            assert ep == o.epoch
            nb += 1
        else:
            rc_o, d_o = o.bfs(it.src)
            rc, d = g.try_bfs(it.src)
            assert rc == rc_o
            if rc == 0:
                assert np.array_equal(d.cpu().numpy(), d_o), ("bfs", nq, it.src)
            nq += 1
    assert nq > 1000 and nb > 1000


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("seed", range(4))
def test_random_batches_all_sizes(dg, seed, undirected):
    """Random op mixes on small graphs, batch sizes from 1 to 4,000, with
    repeated keys inside a batch; all six op types; queries after each batch."""
    n = [9, 40, 300, 2000][seed]
    o = Oracle(n, undirected=undirected, w_max=50)
    g = dg.Graph(n, undirected=undirected, w_max=50)
    say("random batches", seed, undirected)
    load = make_ops([ADDV] * n, np.arange(n), np.zeros(n), np.zeros(n))
    _, r_o = o.apply(load)
    res, _ = g.apply(load)
    assert np.array_equal(res, r_o)
    mix = [0.06, 0.04, 0.05, 0.45, 0.25, 0.15]
    rng = np.random.default_rng(seed)
    for b, size in enumerate([1, 7, 64, 500, 4000, 33, 2]):
        ops = synth.random_ops(n, size, seed * 1000 + b, w_max=50, mix=mix)
        rc_o, r_o = o.apply(ops)
        res, ep = g.apply(ops)
        assert np.array_equal(res, r_o), ("batch", b, np.nonzero(res != r_o)[0][:10])
        assert ep == o.epoch
        check_queries(g, o, ep, rng.integers(0, n, 3), dg, bc=(b % 3 == 2))
    nv, na = g.stats()
    assert (nv, na) == o.counts()


def test_batches_at_the_sort_path_boundary(dg):
    """Batches of 131,072 and 131,073 ops (64 and 65 sort tiles of 2,048
    keys): the first sort sums its offsets inside the scatter, the second
    takes the separate scan; op results and queries equal the oracle's."""
    gr = synth.rmat_graph(13, 8, 50, seed=9)
    o = Oracle(gr.n, w_max=50)
    g = dg.Graph(gr.n, w_max=50)
    say("sort path boundary")
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    mix = [0.02, 0.01, 0.02, 0.45, 0.35, 0.15]
    for b, size in enumerate([131_072, 131_073]):
        ops = synth.random_ops(gr.n, size, 700 + b, w_max=50, mix=mix)
        rc_o, r_o = o.apply(ops)
        res, ep = g.apply(ops)
        assert np.array_equal(res, r_o), ("batch", size, np.nonzero(res != r_o)[0][:10])
        check_queries(g, o, ep, synth.out_degree_sources(gr, 2, synth.rng_for(9, b)), dg)
    assert g.stats() == o.counts()


def test_first_batches_of_fresh_graphs(dg):
    """A graph's first batch of host ops, smaller than the batch scratch's
    minimum size, is staged after that scratch is sized: fresh graphs
    created and destroyed in turn (so device blocks are recycled) all apply
    their first batch exactly."""
    for it in range(40):
        n = [9, 300, 700, 1000][it % 4]
        o = Oracle(n, w_max=50)
        g = dg.Graph(n, w_max=50)
        load = make_ops([ADDV] * n, np.arange(n), np.zeros(n), np.zeros(n))
        _, r_o = o.apply(load)
        res, _ = g.apply(load)
        assert np.array_equal(res, r_o), (it, np.nonzero(res != r_o)[0][:10])
        ops = synth.random_ops(n, 200, 500 + it, w_max=50)
        _, r_o = o.apply(ops)
        res, _ = g.apply(ops)
        assert np.array_equal(res, r_o), (it, np.nonzero(res != r_o)[0][:10])
        del g


def test_device_resident_ops_and_results(dg):
    n = 500
    o = Oracle(n, w_max=9)
    g = dg.Graph(n, w_max=9)
    say("device ops")
    ops = np.concatenate([make_ops([ADDV] * n, np.arange(n), np.zeros(n), np.zeros(n)),
                          synth.random_ops(n, 3000, 5, w_max=9, mix=[0.02, 0.02, 0.01, 0.6, 0.2, 0.15])])
    dops = dg.ops_to_device(ops)
    dres = torch.zeros(len(ops), dtype=torch.uint8, device="cuda")
    _, ep = g.apply(dops, dres)
    torch.cuda.synchronize()
    rc, r_o = o.apply(ops)
    assert np.array_equal(dres.cpu().numpy(), r_o)


def test_rejected_batches_change_nothing(dg):
    g = dg.Graph(8, w_max=10)
    g.apply(make_ops([ADDV, ADDV, ADDE], [0, 1, 0], [0, 0, 1], [0, 0, 3]))
    e0 = g.epoch
    say("rejections")
    for bad, code in [(make_ops([REME, ADDE], [0, 0], [1, 8], [0, 1]), dg.E_VERTEX_RANGE),
                      (make_ops([REME, ADDE], [0, 1], [1, 0], [0, 11]), dg.E_WEIGHT_RANGE),
                      (make_ops([REME, 9], [0, 0], [1, 0], [0, 0]), dg.E_INVALID_ARG)]:
        rc, _, _ = g.try_apply(bad)
        assert rc == code
        assert g.epoch == e0
        # a ContainsEdge is itself a one-op batch and publishes an epoch
        r, e0 = g.contains_edge(0, 1)
        assert r == 1
    # empty batch: no epoch bump
    _, ep = g.apply(make_ops([], [], [], []))
    assert ep == e0


def test_source_absent_and_retired_epochs(dg):
    g = dg.Graph(16, w_max=5, max_resident_epochs=2)
    g.apply(make_ops([ADDV] * 4, range(4), [0] * 4, [0] * 4))        # epoch 1
    say("source absent / retired")
    assert g.try_bfs(9)[0] == dg.E_SOURCE_ABSENT
    assert g.try_sssp(9)[0] == dg.E_SOURCE_ABSENT
    assert g.try_bc([0, 9])[0] == dg.E_SOURCE_ABSENT
    assert g.try_bc([0, 0])[0] == dg.E_INVALID_ARG
    assert g.try_bfs(99)[0] == dg.E_VERTEX_RANGE
    g.apply(make_ops([ADDE], [0], [1], [2]))                          # epoch 2
    g.apply(make_ops([ADDE], [1], [2], [2]))                          # epoch 3
    assert g.try_bfs(0, 1)[0] == dg.E_EPOCH_RETIRED                  # window = {2, 3}
    assert g.try_bfs(0, 4)[0] == dg.E_EPOCH_RETIRED                  # not published
    assert g.bfs(0, 2).cpu().tolist()[:4] == [0, 1, -1, -1]
    pin = g.acquire(2)
    g.apply(make_ops([REMV], [1], [0], [0]))                          # epoch 4
    g.apply(make_ops([ADDE], [2], [3], [2]))                          # epoch 5
    assert g.bfs(0, 2).cpu().tolist()[:4] == [0, 1, -1, -1]          # pinned
    assert g.bfs(0, 3).cpu().tolist()[:4] == [0, 1, 2, -1]
    assert g.bfs(0, 5).cpu().tolist()[:4] == [0, -1, -1, -1]
    assert g.try_bfs(1, 5)[0] == dg.E_SOURCE_ABSENT
    assert g.bfs(1, 3).cpu().tolist()[:4] == [-1, 0, 1, -1]
    g.release(pin)
    assert g.try_bfs(0, 2)[0] == dg.E_EPOCH_RETIRED


def test_snapshots_of_many_epochs_match_oracle_history(dg):
    """Queries and out-degrees on every retained epoch after later batches
    changed the graph (versions born and tombstoned since), compared with the
    oracle's answer recorded when it was at that epoch; then after
    compaction."""
    gr = synth.rmat_graph(12, 8, 30, seed=4)
    o = Oracle(gr.n, w_max=30)
    g = dg.Graph(gr.n, w_max=30, max_resident_epochs=6)
    say("epoch history")
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    wl = synth.update_batches(graph=gr, n_batches=5, n_edge_ops=3000, w_max=30, seed=4)
    srcs = wl.bfs_src[:3]
    hist, degs = {}, {}
    for b in wl.batches:
        rc, r_o = o.apply(b)
        res, ep = g.apply(b)
        assert np.array_equal(res, r_o)
        hist[ep] = {int(s): (o.bfs(int(s))[1], o.sssp(int(s))[1]) for s in srcs}
        degs[ep] = np.array([o.out_degree(v) for v in range(gr.n)], np.int64)
    for compacted in (False, True):
        if compacted:
            g.compact()
        for ep, ans in hist.items():
            assert np.array_equal(g.out_degrees(ep).cpu().numpy().astype(np.int64), degs[ep]), (ep, compacted)
            for s, (bd, sd) in ans.items():
                assert np.array_equal(g.bfs(s, ep).cpu().numpy(), bd), (ep, s, compacted)
                assert np.array_equal(g.sssp(s, ep).cpu().numpy(), sd), (ep, s, compacted)


def test_vertex_remove_readd_inside_batch(dg):
    """RemoveVertex then AddVertex then AddEdge of the same key in one batch:
    the old version must go and a new one (new weight) appear."""
    n = 6
    o = Oracle(n, w_max=9)
    g = dg.Graph(n, w_max=9)
    say("remove/re-add")
    load = make_ops([ADDV] * n + [ADDE, ADDE, ADDE], list(range(n)) + [0, 1, 2], [0] * n + [1, 2, 0],
                    [0] * n + [5, 5, 5])
    o.apply(load)
    g.apply(load)
    seq = make_ops([HASE, REMV, HASE, ADDE, ADDV, ADDE, HASE, ADDE, REME, ADDE, HASV, REMV, ADDV],
                   [0, 1, 0, 0, 1, 0, 0, 1, 0, 0, 1, 2, 2],
                   [1, 0, 1, 1, 0, 1, 1, 2, 1, 1, 0, 0, 0],
                   [0, 0, 0, 3, 0, 7, 0, 4, 0, 8, 0, 0, 0])
    rc, r_o = o.apply(seq)
    res, ep = g.apply(seq)
    assert np.array_equal(res, r_o)
    for s in range(n):
        check_queries(g, o, ep, [s], dg)
    assert g.stats() == o.counts()


def test_bulk_load_spans_many_tiles(dg):
    """R-MAT scale 14 bulk load (hubs with hundreds of buckets, many tiles
    per frontier vertex), directed and undirected, all queries exact."""
    for und in (False, True):
        gr = synth.rmat_graph(14, 16, 255, seed=2, undirected=und)
        o = Oracle(gr.n, undirected=und, w_max=255)
        g = dg.Graph(gr.n, undirected=und, w_max=255)
        say("bulk load scale 14", und)
        rc, r_o = o.apply(synth.load_ops(gr))
        res, _ = g.apply(synth.load_ops(gr))
        assert np.array_equal(res, r_o)
        src = synth.out_degree_sources(gr, 4, synth.rng_for(2, 3))
        check_queries(g, o, g.epoch, src, dg, bc=True)
        # out-degrees, hubs counted tile by tile
        want = np.array([o.out_degree(v) for v in range(gr.n)], np.int64)
        assert want.max() > 32 * 16, "no slab longer than one tile"
        assert np.array_equal(g.out_degrees().cpu().numpy().astype(np.int64), want)
        for T in (16, 32, 64):
            g.set_tuning(chunk_buckets=T, sssp_delta=17 * T)
            check_queries(g, o, g.epoch, src[:1], dg)


def test_bfs_direction_thresholds_sweep(dg):
    """BFS levels do not depend on the direction switches: all top-down
    (every frontier counted small), bottom-up from the first large frontier,
    and the defaults, on a directed and an undirected R-MAT graph, before and
    after a batch of deletions, all equal the oracle's."""
    for und in (False, True):
        gr = synth.rmat_graph(12, 16, 20, seed=13, undirected=und)
        o = Oracle(gr.n, undirected=und, w_max=20)
        g = dg.Graph(gr.n, undirected=und, w_max=20)
        o.apply(synth.load_ops(gr))
        g.apply(synth.load_ops(gr))
        src = [int(s) for s in synth.out_degree_sources(gr, 3, synth.rng_for(13, 1))]
        wl = synth.update_batches(graph=gr, n_batches=1, n_edge_ops=4000, w_max=20, seed=13)
        for phase in range(2):
            if phase:
                o.apply(wl.batches[0])
                g.apply(wl.batches[0])
            want = {s: o.bfs(s)[1] for s in src}
            for alpha, beta in ((4, 24), (1000000, 1), (1, 1000000), (1000000, 1000000)):
                say("bfs thresholds", und, phase, alpha, beta)
                g.set_tuning(alpha=alpha, beta=beta)
                for s in src:
                    assert np.array_equal(g.bfs(s, g.epoch).cpu().numpy(), want[s]), (und, phase, alpha, beta, s)


def test_sssp_bucket_width_sweep(dg):
    """Delta-stepping with bucket widths from 1 (Dijkstra-like, every arc
    heavy but weight-1 ones) through w_max (no heavy arcs) to far above it:
    plain and batched SSSP equal the oracle's Dijkstra at every width."""
    gr = synth.rmat_graph(12, 16, 255, seed=7)
    o = Oracle(gr.n, w_max=255)
    g = dg.Graph(gr.n, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    src = [int(s) for s in synth.out_degree_sources(gr, 3, synth.rng_for(7, 3))]
    want = {s: o.sssp(s)[1] for s in src}
    for delta in (1, 2, 7, 64, 254, 255, 256, 100000):
        say("sssp delta", delta)
        g.set_tuning(sssp_delta=delta, batch_delta=delta)
        for s in src:
            assert np.array_equal(g.sssp(s, g.epoch).cpu().numpy(), want[s]), (delta, s)
        outs = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for _ in src]
        st = g.query_batch([(dg.Q_SSSP, g.epoch, s, out) for s, out in zip(src, outs)])
        assert st == [0] * len(src)
        for s, out in zip(src, outs):
            assert np.array_equal(out.cpu().numpy(), want[s]), ("batched", delta, s)


def test_bc_closed_form_and_overflow(dg):
    n = 9
    g = dg.Graph(n, undirected=True, w_max=1)
    ops = make_ops([ADDV] * n + [ADDE] * (n - 1), list(range(n)) + list(range(n - 1)),
                   [0] * n + list(range(1, n)), [0] * n + [1] * (n - 1))
    g.apply(ops)
    say("bc path")
    b = g.bc(list(range(n))).cpu().numpy()
    assert np.array_equal(b, [2.0 * i * (n - 1 - i) for i in range(n)])
    # chain of 63 diamonds: 2^63 shortest paths overflow int64
    k = 63
    us, vs = [], []
    for i in range(k):
        a, bb, c, d = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        us += [a, a, bb, c]
        vs += [bb, c, d, d]
    nn = 3 * k + 1
    g2 = dg.Graph(nn, w_max=1)
    g2.apply(make_ops([ADDV] * nn + [ADDE] * len(us), list(range(nn)) + us, [0] * nn + vs,
                      [0] * nn + [1] * len(us)))
    assert g2.try_bc([0])[0] == dg.E_OVERFLOW
    assert g2.try_bc([3])[0] == 0
