"""The serving loop: interleaved update batches and queries submitted over
time, checked against the oracle replaying the updates in arrival order;
every query's result equals the same query run alone on its bound epoch."""
import time

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


def run_mix(dg, mem_budget, max_batch, n_req=60, seed=3, query_lanes=2):
    gr = synth.rmat_graph(11, 8, 50, seed=seed)
    g = dg.Graph(gr.n, w_max=50, max_resident_epochs=128)
    g.apply(synth.load_ops(gr))
    e_load = g.epoch
    wl = synth.update_batches(graph=gr, n_batches=n_req, n_edge_ops=400, w_max=50, seed=seed)
    srcs = synth.out_degree_sources(gr, 16, synth.rng_for(seed, 4))
    rng = np.random.default_rng(seed)
    srv = dg.Server(g, mem_budget=mem_budget, max_inflight=64, max_batch=max_batch, query_lanes=query_lanes)
    log = []   # (ticket, kind, payload)
    nu = 0
    for i in range(n_req):
        r = rng.random()
        if r < 0.3:
            t = srv.submit_update(wl.batches[nu])
            log.append((t, "update", nu))
            nu += 1
        elif r < 0.6:
            s = int(srcs[rng.integers(len(srcs))])
            log.append((srv.submit_query(dg.Q_BFS, [s]), "bfs", s))
        elif r < 0.9:
            s = int(srcs[rng.integers(len(srcs))])
            log.append((srv.submit_query(dg.Q_SSSP, [s]), "sssp", s))
        else:
            S = [int(x) for x in rng.choice(srcs, 3, replace=False)]
            log.append((srv.submit_query(dg.Q_BC, S), "bc", tuple(S)))
        time.sleep(float(rng.exponential(0.002)))
    srv.drain()
    stats = srv.stats()
    out = []
    for t, kind, payload in log:
        done, st, ep, lat = srv.poll(t)
        assert done
        if kind == "update":
            buf = np.zeros(len(wl.batches[payload]), np.uint8)
        elif kind == "bc":
            buf = np.zeros(gr.n, np.float64)
        else:
            buf = np.zeros(gr.n, np.int32)
        srv.take(t, buf)
        out.append((kind, payload, st, ep, lat, buf))
    srv.stop()
    return gr, g, e_load, wl, out, stats


def check_against_oracle(dg, gr, g, e_load, wl, out):
    o = Oracle(gr.n, w_max=50)
    o.apply(synth.load_ops(gr))
    assert o.epoch == e_load
    updates = [(p, st, ep, buf) for kind, p, st, ep, lat, buf in out if kind == "update"]
    queries = [(kind, p, st, ep, buf) for kind, p, st, ep, lat, buf in out if kind != "update"]
    # updates commit in arrival order, one epoch each
    for j, (p, st, ep, buf) in enumerate(updates):
        assert st == 0 and ep == e_load + 1 + j
    by_epoch = {}
    for q in queries:
        by_epoch.setdefault(q[3], []).append(q)
    for ep in range(e_load, e_load + len(updates) + 1):
        if ep > e_load:
            p, st, uep, buf = updates[ep - e_load - 1]
            rc, want = o.apply(wl.batches[p])
            assert np.array_equal(buf, want), ("update results", ep)
        for kind, p, st, qep, buf in by_epoch.get(ep, []):
            if kind == "bfs":
                rc, want = o.bfs(p)
            elif kind == "sssp":
                rc, want = o.sssp(p)
            else:
                rc, want = o.bc(list(p))
            assert st == rc, (kind, p, ep, st, rc)
            if rc:
                continue
            if kind == "bc":
                assert not (np.abs(buf - want) > BC_RTOL * np.abs(want)).any(), ("bc", ep)
            else:
                assert np.array_equal(buf, want), (kind, p, ep)
            # the same query alone, on its bound epoch
            if kind == "bfs":
                alone = g.bfs(p, ep).cpu().numpy()
            elif kind == "sssp":
                alone = g.sssp(p, ep).cpu().numpy()
            else:
                alone = g.bc(list(p), ep).cpu().numpy()
            if kind == "bc":
                assert not (np.abs(buf - alone) > BC_RTOL * np.abs(alone)).any()
            else:
                assert np.array_equal(buf, alone)
    assert sum(1 for ep in by_epoch if ep < e_load) == 0


@pytest.mark.parametrize("lanes", [1, 3])
def test_serving_mix_matches_oracle_and_alone(dg, lanes):
    """With one lane, and with three lanes whose launches overlap."""
    say("serving mix, lanes", lanes)
    gr, g, e_load, wl, out, stats = run_mix(dg, mem_budget=1 << 30, max_batch=8, query_lanes=lanes)
    check_against_oracle(dg, gr, g, e_load, wl, out)
    assert stats["completed"] == len(out)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0
    assert stats["queries"] + stats["updates"] == len(out)


def test_serving_admission_under_tiny_budget(dg):
    """A budget of two BFS outputs: queries wait for memory but all finish
    with correct results; a BC output larger than the budget is refused."""
    say("serving tiny budget")
    V = 1 << 11
    gr, g, e_load, wl, out, stats = run_mix(dg, mem_budget=2 * 4 * V, max_batch=4, n_req=30, seed=5)
    # BC needs 8V bytes: larger than... exactly the budget, so it is admitted alone
    check_against_oracle(dg, gr, g, e_load, wl, out)
    g2 = dg.Graph(V, w_max=50)
    srv = dg.Server(g2, mem_budget=4 * V, max_inflight=4, max_batch=4)
    with pytest.raises(dg.DGError) as ei:
        srv.submit_query(dg.Q_BC, [0])
    assert ei.value.status == dg.E_BUSY
    srv.stop()
    with pytest.raises(dg.DGError) as ei:
        dg.Server(g2, query_lanes=5)
    assert ei.value.status == dg.E_INVALID_ARG
