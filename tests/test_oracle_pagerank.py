"""Pins for the oracle's PageRank (CPU only).

Eq. (1) has a plain fixed point: on the live vertices,
(I - d M) pr = (1 - d)/n, with M[u, v] = 1/q(v) for every arc (v, u).  The
pins check the oracle against that linear system solved densely (numpy),
against closed forms (cycles, a single arc, stars, d = 0), against the sum
invariant (sum pr = 1 when no live vertex lacks out-arcs), and against the
stopping rule of the Barrier baseline (Alg. 1): the loop ends at the first
iteration whose largest change is at most the threshold.

Bound used by the dense-solve pin: the iteration is a d-contraction in the
L1 norm (M's columns sum to 1 or 0), so after the stop
|pr - pr*|_1 <= d/(1-d) * |pr_k - pr_(k-1)|_1 <= d/(1-d) * n * threshold,
which is below 1e-13 for the sizes used here.
"""
import numpy as np
import pytest

from oracle import Oracle, OK, E_INVALID_ARG
from paper_2109_09527_amd import synth
from paper_2109_09527_amd.synth import REMV, make_ops

D = 0.85
THR = 1e-16


def load(n, us, vs, undirected=False):
    o = Oracle(n, undirected=undirected, w_max=255)
    us = np.asarray(us, dtype=np.uint32)
    vs = np.asarray(vs, dtype=np.uint32)
    g = synth.Graph(n, us, vs, np.ones(len(us), np.int32), undirected)
    rc, _ = o.apply(synth.load_ops(g))
    assert rc == OK
    return o


def dense_fixed_point(o, d=D):
    """Solve (I - d M) x = (1 - d)/n on the live vertices (dead ones: 0)."""
    n = o.n
    live = np.array([o.alive(v) for v in range(n)])
    nl = int(live.sum())
    us, vs, _ = o.edges()
    arcs = list(zip(us.tolist(), vs.tolist()))
    if o.undirected:
        arcs += [(b, a) for a, b in arcs if a != b]
    q = np.zeros(n)
    for a, _ in arcs:
        q[a] += 1
    M = np.zeros((n, n))
    for a, b in arcs:
        M[b, a] += 1.0 / q[a]
    idx = np.nonzero(live)[0]
    A = np.eye(nl) - d * M[np.ix_(idx, idx)]
    x = np.zeros(n)
    x[idx] = np.linalg.solve(A, np.full(nl, (1 - d) / nl))
    return x


def test_cycle_is_uniform_after_one_iteration():
    for n in (1, 2, 5, 64):
        us = np.arange(n)
        o = load(n, us, (us + 1) % n) if n > 1 else load(1, [0], [0])
        rc, pr, it, ch = o.pagerank()
        assert rc == OK
        assert it == 1 and ch <= THR
        assert np.all(np.abs(pr - 1.0 / n) <= 1e-18)


def test_single_arc_closed_form_and_iterations():
    # a -> b: pr(a) = (1-d)/2, pr(b) = (1-d)/2 + d (1-d)/2.  From 1/2 each:
    # iteration 1 gives (0.075, 0.5), iteration 2 (0.075, 0.13875),
    # iteration 3 repeats it (change 0), so the loop runs three times.
    o = load(2, [0], [1])
    rc, pr, it, ch = o.pagerank()
    assert rc == OK
    assert it == 3 and ch == 0.0
    assert abs(pr[0] - (1 - D) / 2) <= 1e-17
    assert abs(pr[1] - ((1 - D) / 2 + D * (1 - D) / 2)) <= 1e-17


def test_star_closed_form():
    # k leaves -> centre 0; leaves have out-degree 1 and no in-arcs
    for k in (1, 7, 100):
        n = k + 1
        o = load(n, np.arange(1, n), np.zeros(k))
        rc, pr, it, _ = o.pagerank()
        assert rc == OK
        leaf = (1 - D) / n
        assert np.all(np.abs(pr[1:] - leaf) <= 1e-17)
        assert abs(pr[0] - (leaf + D * k * leaf)) <= 1e-15


def test_undamped_is_uniform():
    gr = synth.rmat_graph(6, 4, 255, seed=3)
    o = load(gr.n, gr.u, gr.v)
    rc, pr, it, ch = o.pagerank(damping=0.0)
    assert rc == OK and it <= 2
    assert np.all(np.abs(pr - 1.0 / gr.n) <= 1e-18)


@pytest.mark.parametrize("undirected", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_matches_dense_linear_solve(seed, undirected):
    """Random graphs with vertices lacking out-arcs (and, after removals,
    dead vertices): the oracle equals the dense solve of Eq. (1)."""
    rng = synth.rng_for(seed, 90)
    n = 40
    m = 120
    us = rng.integers(0, n, m)
    vs = rng.integers(0, n, m)
    keep = us != vs
    o = load(n, us[keep], vs[keep], undirected)
    dead = rng.choice(n, 5, replace=False)
    rc, _ = o.apply(make_ops(np.full(len(dead), REMV), dead, np.zeros(len(dead))))
    assert rc == OK
    rc, pr, it, ch = o.pagerank()
    assert rc == OK and ch <= THR
    want = dense_fixed_point(o)
    assert np.all(pr[dead] == 0.0)
    assert np.max(np.abs(pr - want)) <= 1e-13, np.max(np.abs(pr - want))


def test_directed_uses_in_arcs_not_out_arcs():
    # 0 -> 1, 0 -> 2, 1 -> 2: pulling over out-arcs instead would rank 0 highest
    o = load(3, [0, 0, 1], [1, 2, 2])
    _, pr, _, _ = o.pagerank()
    want = dense_fixed_point(o)
    assert np.max(np.abs(pr - want)) <= 1e-15
    assert pr[2] > pr[1] > pr[0]


def test_sum_is_one_without_dangling_vertices():
    gr = synth.rmat_graph(8, 8, 255, seed=5, undirected=True)
    o = load(gr.n, gr.u, gr.v, undirected=True)
    # isolated vertices have no out-arcs; drop them so that none dangles
    iso = [v for v in range(gr.n) if o.out_degree(v) == 0]
    o.apply(make_ops(np.full(len(iso), REMV), np.array(iso), np.zeros(len(iso))))
    rc, pr, it, _ = o.pagerank()
    assert rc == OK
    assert abs(pr.sum() - 1.0) <= 1e-13
    # with dangling vertices mass leaks: the sum is below one
    o2 = load(3, [0], [1])
    assert o2.pagerank()[1].sum() < 1.0


def test_stops_at_first_iteration_within_threshold():
    gr = synth.rmat_graph(7, 8, 255, seed=9)
    o = load(gr.n, gr.u, gr.v)
    rc, pr, it, ch = o.pagerank()
    assert rc == OK and ch <= THR and it > 3
    # one iteration fewer has not yet reached the threshold
    _, _, it2, ch2 = o.pagerank(max_iters=it - 1)
    assert it2 == it - 1 and ch2 > THR
    # a looser threshold stops earlier, at a change within it
    _, _, it3, ch3 = o.pagerank(threshold=1e-8)
    assert it3 < it and ch3 <= 1e-8


def test_empty_and_invalid():
    o = Oracle(5)
    rc, pr, it, ch = o.pagerank()
    assert rc == OK and it == 0 and not pr.any()
    o = load(3, [0], [1])
    assert o.pagerank(damping=1.0)[0] == E_INVALID_ARG
    assert o.pagerank(damping=-0.1)[0] == E_INVALID_ARG
    assert o.pagerank(threshold=-1.0)[0] == E_INVALID_ARG


# ------------------------------------------------------- loop perforation (Alg. 5)

def test_perforation_hand_traced():
    # d = 1/2 on 0 -> 1, 1 -> 2, 2 -> 1, and an isolated 3 (n = 4): every
    # value is a binary fraction, so the trace is exact.  From 1/4 each:
    #   iteration 1: (1/8, 3/8, 1/4, 1/8)
    #   iteration 2: (1/8, 5/16, 5/16, 1/8); vertices 1 and 2 change by 1/16
    #   iteration 3 without perforation: (1/8, 11/32, 9/32, 1/8), on towards
    #   the fixed point (1/8, 1/3, 7/24, 1/8).
    # With freeze_below = 0.07 both freeze after iteration 2 (change 1/16),
    # iteration 3 changes nothing, and the loop stops there.
    o = load(4, [0, 1, 2], [1, 2, 1])
    rc, pr, it, ch = o.pagerank(damping=0.5, freeze_below=0.07)
    assert rc == OK and it == 3 and ch == 0.0
    assert pr.tolist() == [0.125, 0.3125, 0.3125, 0.125]
    _, pr2, it2, _ = o.pagerank(damping=0.5, max_iters=3)
    assert pr2.tolist() == [0.125, 11 / 32, 9 / 32, 0.125]
    _, pr3, _, _ = o.pagerank(damping=0.5)
    assert np.max(np.abs(pr3 - [0.125, 1 / 3, 7 / 24, 0.125])) <= 1e-15


def test_perforation_at_the_papers_scale_stays_exact():
    """With the paper's 1e-21 against a 1e-16 threshold, perforation takes
    no more iterations and moves no rank measurably: the ranks still equal
    the dense solve, and freeze_below = 0 is the plain iteration exactly."""
    for seed, und in ((1, False), (2, True)):
        rng = synth.rng_for(seed, 91)
        n = 40
        us = rng.integers(0, n, 120)
        vs = rng.integers(0, n, 120)
        keep = us != vs
        o = load(n, us[keep], vs[keep], und)
        _, a, ia, _ = o.pagerank(freeze_below=1e-21)
        _, b, ib, _ = o.pagerank()
        _, c, ic, _ = o.pagerank(freeze_below=0.0)
        assert ia <= ib and ic == ib and np.array_equal(b, c)
        assert np.max(np.abs(a - dense_fixed_point(o))) <= 1e-13
    assert load(3, [0], [1]).pagerank(freeze_below=-1.0)[0] == E_INVALID_ARG
