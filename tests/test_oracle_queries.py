"""Pins for the oracle's snapshot queries (CPU only).

BFS: boolean matrix powers, Warshall closure and closed forms.
SSSP: Bellman-Ford rounds, unit weights == BFS, closed forms.
BC: all-pairs path counts from integer matrix powers, closed forms for
paths / stars / complete graphs / cycles, the sum invariant, a hand-derived
fixture, and int64 overflow on a chain of diamonds (sigma = 2^k exactly).
"""
import numpy as np
import pytest

from oracle import Oracle, OK, E_SOURCE_ABSENT, E_OVERFLOW, E_INVALID_ARG
from paper_2109_09527_amd import synth
from paper_2109_09527_amd.synth import ADDV, ADDE, REMV, make_ops
from tests.brute import (MatrixModel, bfs_by_powers, warshall, bellman_ford, bc_brute,
                         bc_sum_rhs)
from tests.golden_io import read_bc_fixture


def load(n, us, vs, ws=None, undirected=False, w_max=255):
    o = Oracle(n, undirected=undirected, w_max=w_max)
    us = np.asarray(us, dtype=np.uint32)
    vs = np.asarray(vs, dtype=np.uint32)
    ws = np.ones(len(us), np.int32) if ws is None else np.asarray(ws, dtype=np.int32)
    g = synth.Graph(n, us, vs, ws, undirected)
    rc, res = o.apply(synth.load_ops(g))
    assert rc == OK
    return o


def dense(n, us, vs, ws=None, undirected=False):
    A = np.zeros((n, n), bool)
    W = np.zeros((n, n), np.int64)
    ws = np.ones(len(us)) if ws is None else ws
    A[us, vs] = True
    W[us, vs] = ws
    if undirected:
        A[vs, us] = True
        W[vs, us] = ws
    return A, W


# ------------------------------------------------------------------ BFS

@pytest.mark.parametrize("n", [1, 2, 7, 30])
def test_bfs_closed_forms(n):
    # directed path 0->1->...->n-1: dist(s, t) = t - s for t >= s
    o = load(n, range(n - 1), range(1, n))
    for s in range(n):
        rc, d = o.bfs(s)
        want = np.array([t - s if t >= s else -1 for t in range(n)])
        assert rc == OK and np.array_equal(d, want)
    # directed cycle: (t - s) mod n
    if n >= 2:
        o = load(n, range(n), [(i + 1) % n for i in range(n)])
        for s in range(n):
            rc, d = o.bfs(s)
            assert np.array_equal(d, (np.arange(n) - s) % n)
    # complete digraph: 1 everywhere but the source
    us, vs = np.nonzero(~np.eye(n, dtype=bool))
    o = load(n, us, vs)
    rc, d = o.bfs(0)
    assert d[0] == 0 and (d[1:] == 1).all()
    # out-star centred at 0: leaves at 1, and a leaf reaches nothing
    o = load(n, [0] * (n - 1), range(1, n))
    assert np.array_equal(o.bfs(0)[1], np.r_[0, np.ones(n - 1, int)])
    if n > 1:
        d = o.bfs(1)[1]
        assert d[1] == 0 and (np.delete(d, 1) == -1).all()


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("undirected", [False, True])
def test_bfs_vs_matrix_powers_and_closure(seed, undirected):
    n = 5 + 4 * seed
    g = synth.random_small_graph(n, 2.0 / n, seed, undirected=undirected)
    o = load(n, g.u, g.v, g.w, undirected, w_max=9)
    A, _ = dense(n, g.u, g.v, g.w, undirected)
    R = warshall(A)
    for s in range(n):
        rc, d = o.bfs(s)
        assert rc == OK
        assert np.array_equal(d, bfs_by_powers(A, s))
        reach = R[s].copy()
        reach[s] = True
        assert np.array_equal(d >= 0, reach)


def test_bfs_source_absent_and_dead_vertices():
    o = load(4, [0, 1, 2], [1, 2, 3])
    rc, _ = o.apply(make_ops([REMV], [2], [0], [0]))
    assert rc == OK
    rc, d = o.bfs(0)
    assert rc == OK and d.tolist() == [0, 1, -1, -1]
    assert o.bfs(2)[0] == E_SOURCE_ABSENT
    assert o.sssp(2)[0] == E_SOURCE_ABSENT
    assert o.bc([0, 2])[0] == E_SOURCE_ABSENT


# ----------------------------------------------------------------- SSSP

@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("undirected", [False, True])
def test_sssp_vs_bellman_ford(seed, undirected):
    n = 6 + 5 * seed
    g = synth.random_small_graph(n, 3.0 / n, seed + 50, w_max=20, undirected=undirected)
    o = load(n, g.u, g.v, g.w, undirected, w_max=20)
    A, W = dense(n, g.u, g.v, g.w, undirected)
    for s in range(0, n, max(1, n // 6)):
        rc, d = o.sssp(s)
        assert rc == OK
        assert np.array_equal(d, bellman_ford(A, W, s))


def test_sssp_unit_weights_equal_bfs_and_path_prefix_sums():
    g = synth.random_small_graph(40, 0.06, 3)
    o = load(40, g.u, g.v)
    for s in range(40):
        assert np.array_equal(o.sssp(s)[1], o.bfs(s)[1])
    w = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.int32)
    o = load(9, range(8), range(1, 9), w, w_max=9)
    assert np.array_equal(o.sssp(0)[1], np.r_[0, np.cumsum(w)])
    # a heavy direct arc loses to a light detour
    o = load(3, [0, 0, 1], [2, 1, 2], [9, 1, 1], w_max=9)
    assert o.sssp(0)[1].tolist() == [0, 1, 2]


def test_golden_adt_scenario_state_sssp_matches_matrix_model():
    ops = synth.random_ops(12, 400, 77, w_max=9, mix=[0.1, 0.03, 0.02, 0.55, 0.2, 0.1])
    o = Oracle(12, w_max=9)
    m = MatrixModel(12)
    o.apply(ops)
    m.apply(ops)
    for s in range(12):
        rc, d = o.sssp(s)
        if m.alive[s]:
            assert rc == OK and np.array_equal(d, bellman_ford(m.A, m.W, s))
        else:
            assert rc == E_SOURCE_ABSENT


# ------------------------------------------------------------------- BC

def test_bc_golden_fixture():
    n, arcs, S, want = read_bc_fixture("diamond_bc.txt")
    o = load(n, arcs[:, 0], arcs[:, 1])
    rc, bc = o.bc(S)
    assert rc == OK
    assert np.allclose(bc, want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("undirected", [False, True])
def test_bc_vs_all_pairs_path_counts(seed, undirected):
    n = 6 + 3 * seed
    g = synth.random_small_graph(n, 2.5 / n, seed + 200, undirected=undirected)
    o = load(n, g.u, g.v, None, undirected)
    A, _ = dense(n, g.u, g.v, None, undirected)
    S = np.random.default_rng(seed).permutation(n)[: max(1, n // 2)]
    rc, bc = o.bc(S)
    assert rc == OK
    want = bc_brute(A, S)
    assert np.allclose(bc, want, rtol=1e-12, atol=1e-12)


def _und(n, edges):
    e = np.array(edges, dtype=np.uint32).reshape(-1, 2)
    return load(n, e[:, 0], e[:, 1], undirected=True)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 11])
def test_bc_closed_forms_undirected(n):
    allv = np.arange(n, dtype=np.uint32)
    # path P_n: BC(i) = 2 i (n-1-i)
    o = _und(n, [(i, i + 1) for i in range(n - 1)])
    assert np.allclose(o.bc(allv)[1], [2 * i * (n - 1 - i) for i in range(n)])
    # star K_{1,n-1}: centre (n-1)(n-2), leaves 0
    o = _und(n, [(0, i) for i in range(1, n)])
    assert np.allclose(o.bc(allv)[1], [(n - 1) * (n - 2)] + [0] * (n - 1))
    # complete graph: 0
    o = _und(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    assert np.allclose(o.bc(allv)[1], 0.0)
    # cycle: odd n = 2k+1 -> k(k-1); even n = 2k -> (k-1)^2
    o = _und(n, [(i, (i + 1) % n) for i in range(n)])
    k = n // 2
    want = k * (k - 1) if n % 2 else (k - 1) ** 2
    assert np.allclose(o.bc(allv)[1], want)


@pytest.mark.parametrize("undirected", [False, True])
def test_bc_sum_invariant_random(undirected):
    g = synth.rmat_graph(10, 8, 1, seed=3, undirected=undirected, unweighted=True)
    o = Oracle(g.n, undirected=undirected, w_max=1)
    assert o.apply(synth.load_ops(g))[0] == OK
    S = synth.out_degree_sources(g, 32, synth.rng_for(3, 9))
    rc, bc = o.bc(S)
    assert rc == OK
    rows = {int(s): o.bfs(int(s))[1] for s in S}
    rhs = bc_sum_rhs(rows)
    assert abs(bc.sum() - rhs) <= 1e-9 * max(rhs, 1)


def test_bc_sigma_overflow_on_diamond_chain():
    """k diamonds in series: sigma at the end is exactly 2^k; k = 62 fits,
    k = 63 overflows int64."""
    def chain(k):
        us, vs = [], []
        for i in range(k):
            a, b, c, d = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
            us += [a, a, b, c]
            vs += [b, c, d, d]
        return load(3 * k + 1, us, vs)
    o = chain(62)
    rc, bc = o.bc([0])
    assert rc == OK
    # the middle vertex of the last diamond carries half of the 2^62 paths
    # to the end through it: delta = 2^61 / 2^62 * 1 = 0.5
    assert bc[3 * 61 + 1] == pytest.approx(0.5)
    o = chain(63)
    assert o.bc([0])[0] == E_OVERFLOW


def test_bc_rejects_repeated_sources():
    o = load(3, [0, 1], [1, 2])
    assert o.bc([0, 0])[0] == E_INVALID_ARG
