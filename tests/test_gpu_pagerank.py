"""Parity of the snapshot PageRank (dg_pagerank) with the CPU oracle.

Both iterate Eq. (1) synchronously (Alg. 1) in FP64 from 1/n until the
largest change is at most the threshold, but they sum in different orders
(the oracle adds prev(v)/q(v) * d arc by arc, the GPU sums contributions per
piece and then multiplies by d).  Ranks must agree within the per-vertex
bound derived in tests/pr_tolerance.py: twice the stopping distance
thr * max(1, n pr(v) / (1 - d)) plus 64 unit roundoffs of |pr(v)|.
Iteration counts agree within one, except where the rounding of the largest
ranks' sums reaches the threshold (the hub case below).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Oracle  # noqa: E402
from paper_2109_09527_amd import synth  # noqa: E402
from paper_2109_09527_amd.synth import REME, REMV, make_ops  # noqa: E402

from tests.pr_tolerance import assert_pr_close  # noqa: E402


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2109_09527_amd import dg as m
    return m


def say(*a):
    print("[case]", *a, flush=True)


def n_live(o):
    return o.counts()[0]


def check(g, o, epoch=None, iters_exact=False, **kw):
    rc_o, want, it_o, ch_o = o.pagerank(**kw)
    assert rc_o == 0
    ep = g.epoch if epoch is None else epoch
    got, it, ch = g.pagerank(ep, **kw)
    got = got.cpu().numpy()
    thr = kw.get("threshold", 1e-16)
    ratio = assert_pr_close(got, want, thr, kw.get("damping", 0.85), n_live(o))
    print("[pr] err/tol %.3g iterations %d vs %d" % (ratio, it, it_o), flush=True)
    if iters_exact:
        assert it == it_o, (it, it_o)
    else:
        assert abs(it - it_o) <= 1, (it, it_o)
    assert (ch <= thr) == (ch_o <= thr)
    return got, it


def build(dg, n, us, vs, undirected=False):
    us = np.asarray(us, dtype=np.uint32)
    vs = np.asarray(vs, dtype=np.uint32)
    gr = synth.Graph(n, us, vs, np.ones(len(us), np.int32), undirected)
    o = Oracle(n, undirected=undirected, w_max=255)
    g = dg.Graph(n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    return g, o


def test_closed_forms(dg):
    say("single arc")
    g, o = build(dg, 2, [0], [1])
    got, it = check(g, o, iters_exact=True)
    assert it == 3
    say("cycle")
    g, o = build(dg, 50, np.arange(50), (np.arange(50) + 1) % 50)
    got, it = check(g, o, iters_exact=True)
    assert it == 1 and np.all(np.abs(got - 1 / 50) <= 1e-18)
    say("undamped")
    gr = synth.rmat_graph(8, 8, 255, seed=4)
    g, o = build(dg, gr.n, gr.u, gr.v)
    got, _ = check(g, o, damping=0.0)
    assert np.all(np.abs(got - 1 / gr.n) <= 1e-18)


def test_hub_spans_many_pieces_and_tiles(dg):
    """A vertex with thousands of in-arcs (many pull pieces, many build
    tiles) next to vertices with one, both directions.  The hub's rank is
    near 0.46, where one ulp is 5.6e-17 and the rounding of its 8,191-term
    sum moves it by several ulps: its change can stay above 1e-16 (and
    cross 1e-15 at an iteration set by rounding) in either summation order.
    At 1e-12 both stop together; at 1e-16 the GPU either stops or runs into
    max_iters, and its values equal the oracle's converged ones either way."""
    n = 1 << 13
    leaves = np.arange(1, n)
    us = np.concatenate([leaves, np.zeros(300)])
    vs = np.concatenate([np.zeros(n - 1), np.arange(1, 301)])
    for und in (False, True):
        say("hub", und)
        g, o = build(dg, n, us, vs, und)
        check(g, o, threshold=1e-12)
        _, want, _, _ = o.pagerank()
        got, it, ch = g.pagerank(max_iters=400)
        assert ch <= 1e-16 or it == 400, (it, ch)
        r = assert_pr_close(got.cpu().numpy(), want, 1e-16, 0.85, n_live(o), "hub")
        print("[pr] hub err/tol %.3g" % r, flush=True)


@pytest.mark.parametrize("undirected", [False, True])
def test_rmat_snapshots_across_updates(dg, undirected):
    """R-MAT scale 13: PageRank of the load epoch and of the epoch after a
    batch of edge and vertex changes, both read after the second batch
    (snapshot consistency), equal to the oracle's at each state."""
    gr = synth.rmat_graph(13, 16, 255, seed=11, undirected=undirected)
    o = Oracle(gr.n, undirected=undirected, w_max=255)
    g = dg.Graph(gr.n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    e1 = g.acquire()
    want1 = o.pagerank()
    n1 = n_live(o)
    # edge adds and removals of existing edges, vertex removals and re-adds
    rng = synth.rng_for(11, 5)
    pick = rng.choice(gr.m, 2000, replace=False)
    dead = rng.choice(gr.n, 40, replace=False)
    ops = np.concatenate([
        synth.random_ops(gr.n, 3000, 11, w_max=255, mix=[0.02, 0, 0, 0.98, 0, 0]),
        make_ops(np.full(len(pick), REME), gr.u[pick], gr.v[pick]),
        make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead))),
    ])
    ops = ops[rng.permutation(len(ops))]
    rc, r_o = o.apply(ops)
    res, _ = g.apply(ops)
    assert np.array_equal(res, r_o)
    say("rmat13 latest", undirected)
    check(g, o)
    say("rmat13 earlier epoch", undirected)
    got1, it1, _ = g.pagerank(e1)
    r = assert_pr_close(got1.cpu().numpy(), want1[1], 1e-16, 0.85, n1, "earlier epoch")
    print("[pr] earlier epoch err/tol %.3g iterations %d vs %d" % (r, it1, want1[2]), flush=True)
    assert abs(it1 - want1[2]) <= 1
    g.release(e1)


def test_iteration_cap_threshold_and_determinism(dg):
    gr = synth.rmat_graph(12, 16, 255, seed=13)
    g, o = build(dg, gr.n, gr.u, gr.v)
    say("max_iters 5")
    got, it = check(g, o, max_iters=5, iters_exact=True)
    assert it == 5
    say("max_iters 60 (several host batches)")
    check(g, o, max_iters=60, iters_exact=True)
    say("threshold 1e-9")
    check(g, o, threshold=1e-9)
    say("determinism")
    a, ia, _ = g.pagerank()
    b, ib, _ = g.pagerank()
    assert ia == ib and torch.equal(a, b)


def test_degenerate_and_invalid(dg):
    g = dg.Graph(16, w_max=255)
    pr, it, ch = g.pagerank()
    assert it == 0 and not pr.cpu().numpy().any()
    g, o = build(dg, 4, [0, 1], [1, 2])
    pr, it, ch = g.pagerank(max_iters=0)
    assert it == 0 and not pr.cpu().numpy().any()
    pr, it, ch = g.pagerank(threshold=1.0)
    assert it == 0 and not pr.cpu().numpy().any()
    for kw in ({"damping": 1.0}, {"damping": -0.5}, {"threshold": -1.0}, {"threshold": float("nan")}):
        rc, _, _, _ = g.try_pagerank(**kw)
        assert rc == dg.E_INVALID_ARG, kw
    # vertex 3 is live and isolated: (1 - d)/n
    check(g, o, iters_exact=True)


# ------------------------------------------------------------ No-Sync (Alg. 3)

def check_nosync(g, o, epoch=None, **kw):
    """No-Sync stops when every workgroup's last published change is within
    the threshold; its ranks then meet the same tolerance against the
    synchronous oracle's (Lemma 2 of the paper: identical within the
    threshold at the stop)."""
    _, want, it_o, _ = o.pagerank(**kw)
    ep = g.epoch if epoch is None else epoch
    got, sweeps, ch = g.pagerank(ep, nosync=True, **kw)
    got = got.cpu().numpy()
    thr = kw.get("threshold", 1e-16)
    r = assert_pr_close(got, want, thr, kw.get("damping", 0.85), n_live(o), "nosync")
    print("[pr] nosync err/tol %.3g sweeps %d (synchronous iterations %d)" % (r, sweeps, it_o), flush=True)
    assert ch <= thr and sweeps >= 1, (sweeps, ch)
    return got, sweeps, float(np.abs(got - want).sum())


def test_nosync_closed_forms_and_cap(dg):
    say("nosync cycle")
    g, o = build(dg, 50, np.arange(50), (np.arange(50) + 1) % 50)
    got, sweeps, _ = check_nosync(g, o)
    assert np.all(np.abs(got - 1 / 50) <= 1e-18)
    say("nosync single arc")
    g, o = build(dg, 2, [0], [1])
    check_nosync(g, o)
    say("nosync sweep cap")
    gr = synth.rmat_graph(12, 16, 255, seed=13)
    g, o = build(dg, gr.n, gr.u, gr.v)
    _, sweeps, ch = g.pagerank(nosync=True, max_iters=3)
    assert sweeps <= 3 and ch > 1e-16
    say("nosync empty")
    g = dg.Graph(16, w_max=255)
    pr, sweeps, _ = g.pagerank(nosync=True)
    assert sweeps == 0 and not pr.cpu().numpy().any()
    rc, _, _, _ = g.try_pagerank(damping=1.5, nosync=True)
    assert rc == dg.E_INVALID_ARG


@pytest.mark.parametrize("undirected", [False, True])
def test_nosync_rmat_matches_synchronous(dg, undirected):
    """R-MAT scale 14 with a hub-heavy in-degree spread, after a batch of
    removals: No-Sync equals the synchronous oracle within the tolerance,
    on the latest and on a pinned earlier epoch, run after run."""
    gr = synth.rmat_graph(14, 16, 255, seed=17, undirected=undirected)
    o = Oracle(gr.n, undirected=undirected, w_max=255)
    g = dg.Graph(gr.n, undirected=undirected, w_max=255)
    o.apply(synth.load_ops(gr))
    g.apply(synth.load_ops(gr))
    e1 = g.acquire()
    want1 = o.pagerank()[1]
    n1 = n_live(o)
    rng = synth.rng_for(17, 5)
    pick = rng.choice(gr.m, 3000, replace=False)
    ops = make_ops(np.full(len(pick), REME), gr.u[pick], gr.v[pick])
    o.apply(ops)
    g.apply(ops)
    for rep in range(2):
        say("nosync rmat14", undirected, rep)
        _, sweeps, l1 = check_nosync(g, o)
        print("[nosync] sweeps", sweeps, "L1 vs synchronous", l1, flush=True)
    got1, _, ch = g.pagerank(e1, nosync=True)
    assert_pr_close(got1.cpu().numpy(), want1, 1e-16, 0.85, n1, "nosync earlier epoch")
    g.release(e1)


# ------------------------------------------------------- loop perforation (Alg. 5)

def test_perforation_hand_traced_exact(dg):
    """The oracle's hand-traced case (d = 1/2, binary fractions throughout):
    with freeze_below = 0.07 vertices 1 and 2 freeze after iteration 2 and
    the loop stops after iteration 3, in both forms, bit for bit."""
    g, o = build(dg, 4, [0, 1, 2], [1, 2, 1])
    for nosync in (False, True):
        say("perforation hand trace", nosync)
        pr, it, ch = g.pagerank(damping=0.5, freeze_below=0.07, nosync=nosync)
        assert pr.cpu().numpy().tolist() == [0.125, 0.3125, 0.3125, 0.125], nosync
        assert it == 3 and ch == 0.0
    rc, _, _, _ = g.try_pagerank(freeze_below=-1.0)
    assert rc == dg.E_INVALID_ARG


@pytest.mark.parametrize("undirected", [False, True])
def test_perforation_papers_setting(dg, undirected):
    """freeze_below = 1e-21 with threshold 1e-16 (the paper's setting) on
    R-MAT 13: both forms stay within the tolerance of the oracle's
    perforated ranks, and the synchronous form takes about as many
    iterations."""
    gr = synth.rmat_graph(13, 16, 255, seed=19, undirected=undirected)
    g, o = build(dg, gr.n, gr.u, gr.v, undirected)
    say("perforation 1e-21", undirected)
    _, want, it_o, _ = o.pagerank(freeze_below=1e-21)
    for nosync in (False, True):
        got, it, ch = g.pagerank(freeze_below=1e-21, nosync=nosync)
        r = assert_pr_close(got.cpu().numpy(), want, 1e-16, 0.85, n_live(o), ("perforated", nosync))
        print("[pr] perforated nosync=%d err/tol %.3g iterations %d vs %d" % (nosync, r, it, it_o), flush=True)
        assert ch <= 1e-16
        if not nosync:
            assert abs(it - it_o) <= 1, (it, it_o)
