"""Benchmark of the snapshot-query dynamic graph on one MI355X.

Workload (one "step" = one pass of the hot path over one batch):
  R-MAT scale 20 (1,048,576 vertices, 16.8M sampled directed edges with
  a=0.57 b=0.19 c=0.19 d=0.05, repeated keys and self-loops dropped), int32
  weights uniform in [1, 255], bulk-loaded before timing.  Each step applies
  one update batch of 65,536 edge ops (half AddEdge with fresh R-MAT
  endpoints, half RemoveEdge of generated edges) plus 656 vertex ops (half
  AddVertex, half RemoveVertex), shuffled, publishing one epoch; then one
  snapshot BFS and one delta-stepping SSSP from sources drawn among vertices
  with an initial out-arc, on that epoch.

Batched leg (the batched configuration as stated): R-MAT scale 21 (2.1M
vertices, 33.5M sampled edges), loaded as the first snapshot, then 7
batches of log-uniform [65,536, 1,048,576] edge ops (half AddEdge, half
RemoveEdge), one snapshot each; 512 BFS/SSSP queries (query i a BFS when i
is even, bound to snapshot i mod 8) run as one dg_query_batch call against
512 plain calls, outputs compared element by element.

Reported value: snapshot-query GTEPS of the whole job = sum over the
queries of the edges in the traversed component (visible out-degree summed
over reached vertices) / wall time of all timed steps (updates included).
Also: updates/s, query-only GTEPS, p50/p99 latencies, the dominant
kernel's achieved bandwidth against the HBM roofline (HIP events inside
the library, on the stream the kernels run on), and the CPU oracle timed on
a sample of the same steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per visible arc examined, by kernel family:
#   sssp_relax    dst 4 + weight 4 + stamp 8 + dist 4 (atomicMin target)
#   bfs_top_down  dst 4 + stamp 8 + dist 4
#   bfs_bottom_up src 4 + stamp 8 (frontier bit test stays in L2)
BYTES_PER_ARC = {"sssp_relax": 20, "bfs_top_down": 16, "bfs_bottom_up": 12}
# The engine's multi-source BFS (same-snapshot BFS queries share one scan,
# one bit per query): per visible arc dst 4 + stamp 8 + the target's visited
# mask 8 + its next-level mask 8 (read, then atomicOr when it gains bits).
# Its multi-source SSSP (up to 16 same-snapshot queries share one scan, a
# vertex's 16 distances in one line): per arc scanned dst 4 + weight 4 +
# stamp 8, plus per relaxation (arc, query) the target's distance 4.
BATCH_BYTES_PER_ARC = {"batch_bfs": 28}
MS_SSSP_BYTES = {"per_scan": 16, "per_relaxation": 4}
ORACLE_WORKERS_MAX = 16   # the host cores one GPU's share of the box offers
METRIC = "snapshot-query GTEPS + updates/s; p50/p99 query latency, batched vs plain"
# HBM bytes per launch measured with rocprofv3 counters (profiles/*_traffic.txt),
# valid only while the kernel's sources are unchanged (their digest is stored
# beside the figure).
PROFILES = os.path.join(ROOT, "profiles")


def measured_traffic(kernel, workload):
    """Per-launch HBM bytes of `kernel` on `workload` (a file name part, e.g.
    "rmat20") from the committed counter summaries, or None when there is
    none or the kernel's sources changed since."""
    import glob
    from paper_2109_09527_amd.rocprof_summary import sources_digest
    for path in sorted(glob.glob(os.path.join(PROFILES, f"*_{workload}_traffic.txt"))):
        try:
            with open(path) as f:
                recs = [json.loads(line[5:]) for line in f if line.startswith("json:")]
        except (OSError, ValueError):
            continue
        for rec in recs:
            if rec.get("kernel") != kernel or "sources" not in rec:
                continue
            try:
                if sources_digest([os.path.join(ROOT, p) for p in rec["sources"]]) != rec.get("sources_sha256"):
                    return None
            except OSError:
                return None
            return rec["bytes_per_dispatch"]
    return None


def pct(xs, p):
    """Nearest-rank percentile."""
    xs = sorted(xs)
    if not xs:
        return None
    k = max(1, int(np.ceil(p / 100.0 * len(xs))))
    return xs[k - 1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=6, help="oracle sample size in steps (0 = skip)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, one plain device copy of this many MiB (a reference kernel for "
                         "calibrating HBM byte counters)")
    ap.add_argument("--tuning-file", default=None,
                    help="JSON tuning: loaded (and the autotuner skipped) if the file exists, else written "
                         "after autotuning, so a profiled run can replay the tuned configuration")
    ap.add_argument("--batch-queries", type=int, default=512,
                    help="queries of the batched-vs-plain comparison (0 = skip)")
    ap.add_argument("--batch-scale", type=int, default=21, help="R-MAT scale of the batched comparison")
    ap.add_argument("--batch-tuning-file", default=None,
                    help="as --tuning-file, for the batched comparison's graph")
    ap.add_argument("--tuning", default=None,
                    help="JSON tuning given inline (the autotuner is skipped), e.g. for a profiled run")
    ap.add_argument("--batch-tuning", default=None, help="as --tuning, for the batched comparison's graph")
    ap.add_argument("--c3-oracle", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.c3_oracle:
        # the oracle leg of the batched configuration, in a process of its
        # own that never touches the GPU (its workers are forked from it)
        c3_oracle_child(args.c3_oracle)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the store and its queries run on a single GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2109_09527_amd import dg, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    K, W = args.steps, args.warmup
    n_batches = K + W
    t0 = time.time()
    wl = synth.update_batches(scale=args.scale, n_batches=n_batches, seed=0)
    gr = wl.graph
    print(f"[bench] workload generated in {time.time() - t0:.1f}s: V={gr.n} m={gr.m}", file=sys.stderr, flush=True)

    g = dg.Graph(gr.n, w_max=255, max_resident_epochs=n_batches + 4, edge_capacity=2 * gr.m)
    load = synth.load_ops(gr)
    t0 = time.time()
    dload = dg.ops_to_device(load)
    dres = torch.empty(len(load), dtype=torch.uint8, device="cuda")
    g.apply(dload, dres)
    torch.cuda.synchronize()
    print(f"[bench] bulk load of {len(load)} ops in {time.time() - t0:.2f}s", file=sys.stderr, flush=True)
    del dload, dres

    dbatches = [dg.ops_to_device(b) for b in wl.batches]
    dresults = [torch.empty(len(b), dtype=torch.uint8, device="cuda") for b in wl.batches]
    dist_b = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for _ in range(n_batches)]
    dist_s = [torch.empty(gr.n, dtype=torch.int32, device="cuda") for _ in range(n_batches)]
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    marks = []
    epochs = []

    def step(i):
        e0, e1, e2, e3 = ev(), ev(), ev(), ev()
        e0.record()
        _, ep = g.apply(dbatches[i], dresults[i])
        e1.record()
        g.bfs(int(wl.bfs_src[i]), ep, dist_b[i])
        e2.record()
        g.sssp(int(wl.sssp_src[i]), ep, dist_s[i])
        e3.record()
        return ep, (e0, e1, e2, e3)

    fixed_tuning = bool(args.tuning or (args.tuning_file and os.path.exists(args.tuning_file)))
    if args.tuning:
        g.set_tuning(**json.loads(args.tuning))
    elif fixed_tuning:
        with open(args.tuning_file) as f:
            g.set_tuning(**json.load(f))
    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    if fixed_tuning:
        tuning = g.get_tuning()
    else:
        tuning = g.autotune(seed=0) if not args.no_autotune else g.get_tuning()
        if args.tuning_file:
            with open(args.tuning_file, "w") as f:
                json.dump(tuning, f)
    print(f"[bench] tuning {tuning}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if not args.no_profile:
        g.profile(True)
        g.profile_read(reset=True)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()   # no collector pause of this interpreter inside a timed region
    t_start = time.perf_counter()
    for i in range(W, W + K):
        ep, m = step(i)
        epochs.append(ep)
        marks.append(m)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    gc.enable()
    prof = g.profile_read(reset=True) if not args.no_profile else {}
    g.profile(False)

    upd_ms = [a.elapsed_time(b) for a, b, _, _ in marks]
    bfs_ms = [b.elapsed_time(c) for _, b, c, _ in marks]
    sssp_ms = [c.elapsed_time(d) for _, _, c, d in marks]

    # TEPS numerators: visible out-degree summed over reached vertices
    m_bfs, m_sssp = [], []
    for j, i in enumerate(range(W, W + K)):
        deg = g.out_degrees(epochs[j]).to(torch.int64)
        m_bfs.append(int(deg[dist_b[i] >= 0].sum().item()))
        m_sssp.append(int(deg[dist_s[i] >= 0].sum().item()))
    m_total = sum(m_bfs) + sum(m_sssp)
    n_ops = sum(len(wl.batches[i]) for i in range(W, W + K))
    value = m_total / t_total / 1e9
    q_time = (sum(bfs_ms) + sum(sssp_ms)) / 1e3

    roof = None
    if prof:
        cands = [(v["total_ms"], k) for k, v in prof.items() if k in BYTES_PER_ARC]
        if cands:
            _, kname = max(cands)
            kp = prof[kname]
            avg_ms = kp["total_ms"] / kp["launches"]
            bytes_per_launch = kp["arcs"] * BYTES_PER_ARC[kname] / kp["launches"]
            achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
            traffic = measured_traffic("k_" + kname, "rmat20")
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                    "avg_launch_us": round(avg_ms * 1e3, 2), "launches": kp["launches"],
                    "bytes_per_launch": int(bytes_per_launch)}

    cpu = None
    if args.cpu_steps > 0:
        cpu = cpu_baseline(wl, W, min(args.cpu_steps, K), m_bfs, m_sssp, dist_b, dist_s)

    # the batched configuration runs on a graph of its own
    g.close()
    del dbatches, dresults, dist_b, dist_s
    torch.cuda.empty_cache()
    batched = None
    if args.batch_queries > 0:
        batched, c3_cpu = batched_vs_plain(args)
        if cpu is not None and c3_cpu is not None:
            cpu["batched_config"] = c3_cpu

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(t_total / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"R-MAT scale {args.scale} dynamic graph: per step one batch of 65,536 edge add/remove "
                        f"(50/50) + 656 vertex add/remove, then one snapshot BFS and one delta-stepping SSSP",
            "vertices": gr.n, "loaded_edges": gr.m, "weights": "int32 U[1,255]",
            "ops_per_batch": len(wl.batches[0]), "parallelism": "single GPU", "tuning": tuning,
        },
        "updates_per_s": round(n_ops / (sum(upd_ms) / 1e3), 1),
        "query_gteps": round(m_total / q_time / 1e9, 4),
        "latency_ms": {
            "update_p50": round(pct(upd_ms, 50), 3), "update_p99": round(pct(upd_ms, 99), 3),
            "bfs_p50": round(pct(bfs_ms, 50), 3), "bfs_p99": round(pct(bfs_ms, 99), 3),
            "sssp_p50": round(pct(sssp_ms, 50), 3), "sssp_p99": round(pct(sssp_ms, 99), 3),
        },
        "kernels": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3), "arcs": v["arcs"]}
                    for k, v in prof.items()},
        "roofline": roof,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.copy_mib > 0:
        n = args.copy_mib << 18   # int32 elements
        a = torch.ones(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copied {args.copy_mib} MiB device to device", file=sys.stderr, flush=True)


def kernel_roof(prof, name, bytes_per_arc):
    kp = prof.get(name)
    if not kp or not kp["launches"] or kp["total_ms"] <= 0:
        return None
    achieved = kp["arcs"] * bytes_per_arc / (kp["total_ms"] / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": name,
            "avg_launch_us": round(kp["total_ms"] / kp["launches"] * 1e3, 2), "launches": kp["launches"],
            "bytes_per_launch": int(kp["arcs"] * bytes_per_arc / kp["launches"])}


def batched_vs_plain(args):
    """The batched configuration: R-MAT scale 21 loaded as the first of 8
    snapshots, 7 batches of log-uniform [64k, 1M] edge ops, 512 BFS/SSSP
    queries as one dg_query_batch call against one plain call per query.
    Outputs of the two forms are compared element by element; the oracle is
    then timed on a sample of the same queries, single-threaded and on the
    host's cores."""
    import hashlib

    import torch
    from paper_2109_09527_amd import dg, synth
    t0 = time.time()
    eq = synth.epoch_queries(scale=args.batch_scale, n_queries=args.batch_queries, seed=0)
    gr = eq.graph
    g = dg.Graph(gr.n, w_max=255, max_resident_epochs=8, edge_capacity=2 * gr.m)
    load = synth.load_ops(gr)
    g.apply(dg.ops_to_device(load), torch.empty(len(load), dtype=torch.uint8, device="cuda"))
    epochs = [g.epoch]
    for b in eq.batches:
        _, ep = g.apply(dg.ops_to_device(b), torch.empty(len(b), dtype=torch.uint8, device="cuda"))
        epochs.append(ep)
    torch.cuda.synchronize()
    print(f"[bench] batched configuration: R-MAT {args.batch_scale}, m={gr.m}, batches "
          f"{[len(b) for b in eq.batches]}, ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    tf = args.batch_tuning_file
    if args.batch_tuning:
        g.set_tuning(**json.loads(args.batch_tuning))
        tuning = g.get_tuning()
    elif tf and os.path.exists(tf):
        with open(tf) as f:
            g.set_tuning(**json.load(f))
        tuning = g.get_tuning()
    else:
        tuning = g.autotune(seed=0)
        if tf:
            with open(tf, "w") as f:
                json.dump(tuning, f)
    print(f"[bench] batched configuration tuning {tuning}", file=sys.stderr, flush=True)
    n = gr.n
    nq = len(eq.kinds)
    qs = [(dg.Q_BFS if eq.kinds[i] == 0 else dg.Q_SSSP, epochs[eq.epoch_slot[i]], int(eq.src[i])) for i in range(nq)]
    plain = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in qs]
    batch = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in qs]
    # warm-up of both forms; the engine's warm-up runs the whole batch, so
    # its scratch (sized by the batch) is allocated before the clock starts
    g.query_batch([(k, e, s, o) for (k, e, s), o in zip(qs, batch)])
    for (k, e, s), o in zip(qs[:2], plain[:2]):
        (g.bfs if k == dg.Q_BFS else g.sssp)(s, e, o)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    lat = []
    t0 = time.perf_counter()
    for (k, e, s), o in zip(qs, plain):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        (g.bfs if k == dg.Q_BFS else g.sssp)(s, e, o)
        b.record()
        lat.append((a, b))
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain_ms = [a.elapsed_time(b) for a, b in lat]
    g.profile(True)
    g.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.query_batch([(k, e, s, o) for (k, e, s), o in zip(qs, batch)])
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    gc.enable()
    prof = g.profile_read(reset=True)
    g.profile(False)
    same = all(x == 0 for x in st) and all(torch.equal(a, b) for a, b in zip(plain, batch))
    degs = {e: g.out_degrees(e).to(torch.int64) for e in set(epochs)}
    ms = [int(degs[e][o >= 0].sum().item()) for (k, e, s), o in zip(qs, batch)]
    m = sum(ms)
    roof = {k: kernel_roof(prof, k, BATCH_BYTES_PER_ARC[k]) for k in BATCH_BYTES_PER_ARC}
    if roof.get("batch_bfs"):
        # one launch is one level's expansion of a multi-source BFS group
        roof["batch_bfs"]["kernel"] = "k_mf_pass"
        roof["batch_bfs"]["traffic"] = measured_traffic("k_mf_pass", f"rmat{args.batch_scale}")
    kp, sc = prof.get("batch_sssp"), prof.get("batch_sssp_scan")
    if kp and sc and kp["launches"] and kp["total_ms"] > 0:
        nbytes = MS_SSSP_BYTES["per_scan"] * sc["arcs"] + MS_SSSP_BYTES["per_relaxation"] * kp["arcs"]
        achieved = nbytes / (kp["total_ms"] / 1e3) / 1e9
        roof["batch_sssp"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(achieved / HBM_PEAK_GBS, 4),
                              "traffic": measured_traffic("k_ms_relax", f"rmat{args.batch_scale}"), "kernel": "k_ms_relax",
                              "avg_launch_us": round(kp["total_ms"] / kp["launches"] * 1e3, 2),
                              "launches": kp["launches"], "bytes_per_launch": int(nbytes / kp["launches"]),
                              "arcs_scanned": sc["arcs"], "relaxations": kp["arcs"],
                              "queries_per_scan": round(kp["arcs"] / max(1, sc["arcs"]), 2)}
    out = {"config": {"workload": f"R-MAT scale {args.batch_scale}: {nq} snapshot BFS/SSSP queries (50/50) over "
                                  f"{len(epochs)} epochs (load + batches of log-uniform 64k-1M edge ops), one "
                                  f"persistent batched call vs {nq} plain calls",
                      "vertices": n, "loaded_edges": gr.m, "batch_ops": [len(b) for b in eq.batches],
                      "tuning": tuning},
           "queries": nq, "epochs": len(set(epochs)), "plain_s": round(t_plain, 4), "batched_s": round(t_batch, 4),
           "plain_gteps": round(m / t_plain / 1e9, 4), "batched_gteps": round(m / t_batch / 1e9, 4),
           "speedup": round(t_plain / t_batch, 2),
           "plain_latency_ms": {"p50": round(pct(plain_ms, 50), 3), "p99": round(pct(plain_ms, 99), 3)},
           "batched_latency_ms": {"p50": round(t_batch * 1e3, 3), "p99": round(t_batch * 1e3, 3)},
           "outputs_equal": same,
           "kernels": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3), "arcs": v["arcs"]}
                       for k, v in prof.items()},
           "roofline": roof}
    cpu = None
    if args.cpu_steps > 0:
        # the oracle sample: the first 2 queries of each epoch single-threaded,
        # the first 16 of each epoch on the host's cores
        by_epoch = {}
        for i in range(nq):
            by_epoch.setdefault(int(eq.epoch_slot[i]), []).append(i)
        single = [i for k in sorted(by_epoch) for i in by_epoch[k][:2]]
        par = [i for k in sorted(by_epoch) for i in by_epoch[k][:16]]
        want = {i: hashlib.sha256(batch[i].cpu().numpy().tobytes()).hexdigest() for i in set(single) | set(par)}
        g.close()
        del plain, batch
        torch.cuda.empty_cache()
        cpu = c3_oracle_leg(args, single, par, ms, want)
    return out, cpu


def cpu_info():
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def c3_oracle_leg(args, single, par, ms, want):
    """Runs the oracle on the batched configuration's sample in a child
    process (it never initialises the GPU, so it may fork workers)."""
    import subprocess
    import tempfile
    job = {"scale": args.batch_scale, "n_queries": args.batch_queries, "single": single, "parallel": par,
           "m": {str(i): ms[i] for i in set(single) | set(par)}}
    with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
        json.dump(job, f)
        path = f.name
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--c3-oracle", path], capture_output=True,
                           text=True, timeout=600)
    finally:
        os.unlink(path)
    sys.stderr.write(r.stderr)
    if r.returncode != 0:
        return {"error": f"oracle leg exited with {r.returncode}"}
    res = json.loads(r.stdout.strip().splitlines()[-1])
    hashes = res.pop("hashes")
    res["matches_gpu"] = all(hashes.get(str(i)) == want[i] for i in want)
    return res


def _c3_worker(args):
    """A forked worker: one query on the oracle state inherited at fork."""
    import hashlib
    kind, s = args
    t = time.perf_counter()
    _, d = (_ORC.bfs if kind == 0 else _ORC.sssp)(s)
    return time.perf_counter() - t, hashlib.sha256(d.tobytes()).hexdigest()


_ORC = None


def c3_oracle_child(path):
    """Oracle timing of the batched configuration: the oracle replays the
    load and the batches in order; at each epoch it runs that epoch's
    single-threaded sample one query after another on one core, then its
    parallel sample on up to 16 forked workers.  GTEPS use the GPU's TEPS
    numerators (passed in), which the output hashes tie to these runs."""
    global _ORC
    import multiprocessing as mp

    from oracle import Oracle
    from paper_2109_09527_amd import synth
    with open(path) as f:
        job = json.load(f)
    t0 = time.time()
    eq = synth.epoch_queries(scale=job["scale"], n_queries=job["n_queries"], seed=0)
    gr = eq.graph
    o = Oracle(gr.n, w_max=255)
    o.apply(synth.load_ops(gr))
    print(f"[bench] oracle load of R-MAT {job['scale']} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    single, par = set(job["single"]), set(job["parallel"])
    cpus = sorted(os.sched_getaffinity(0))
    workers = max(1, min(ORACLE_WORKERS_MAX, len(cpus)))
    t_single = 0.0
    m_single = 0
    t_par = 0.0
    m_par = 0
    hashes = {}
    _ORC = o
    ctx = mp.get_context("fork")
    for k in range(len(eq.batches) + 1):
        if k > 0:
            o.apply(eq.batches[k - 1])
        idx = [i for i in range(job["n_queries"]) if int(eq.epoch_slot[i]) == k]
        mine = [i for i in idx if i in single]
        os.sched_setaffinity(0, {cpus[0]})
        for i in mine:
            dt, h = _c3_worker((int(eq.kinds[i]), int(eq.src[i])))
            t_single += dt
            m_single += job["m"][str(i)]
            hashes[str(i)] = h
        os.sched_setaffinity(0, set(cpus))
        mine = [i for i in idx if i in par]
        if mine:
            t = time.perf_counter()
            with ctx.Pool(workers) as pool:
                res = pool.map(_c3_worker, [(int(eq.kinds[i]), int(eq.src[i])) for i in mine], chunksize=1)
            t_par += time.perf_counter() - t
            for i, (_, h) in zip(mine, res):
                m_par += job["m"][str(i)]
                if hashes.setdefault(str(i), h) != h:
                    hashes[str(i)] = "mismatch"
    model, nproc, affinity = cpu_info()
    print(json.dumps({
        "single_thread": {"value": round(m_single / t_single / 1e9, 5), "unit": "GTEPS", "cores": 1,
                          "queries": len(single), "seconds": round(t_single, 2)},
        "parallel": {"value": round(m_par / t_par / 1e9, 5), "unit": "GTEPS", "cores": workers,
                     "queries": len(par), "seconds": round(t_par, 2),
                     "how": "independent queries on forked worker processes, each the plain sequential oracle; "
                            "wall time per epoch includes forking the pool"},
        "sample": "the batched configuration's queries: the first 2 of each epoch single-threaded (pinned to one "
                  "core), the first 16 of each epoch on the parallel workers",
        "cpu_model": model, "nproc": nproc, "affinity_cpus": affinity,
        "hashes": hashes}), flush=True)


def cpu_baseline(wl, W, S, m_bfs, m_sssp, dist_b, dist_s):
    """The sequential oracle on the host: load and the W warm-up batches
    untimed, then S steps (batch + BFS + SSSP) timed with the same metric.
    Its outputs are also compared with the GPU's for those steps."""
    from oracle import Oracle
    gr = wl.graph
    o = Oracle(gr.n, w_max=255)
    t0 = time.time()
    o.apply(synth_load(gr))
    for i in range(W):
        o.apply(wl.batches[i])
    print(f"[bench] oracle setup {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    same = True
    t = 0.0
    cpus = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {cpus[0]})   # single-threaded on one core
    for j in range(S):
        i = W + j
        t1 = time.perf_counter()
        o.apply(wl.batches[i])
        _, db = o.bfs(int(wl.bfs_src[i]))
        _, ds = o.sssp(int(wl.sssp_src[i]))
        t += time.perf_counter() - t1
        same &= bool(np.array_equal(db, dist_b[i].cpu().numpy()) and np.array_equal(ds, dist_s[i].cpu().numpy()))
    os.sched_setaffinity(0, set(cpus))
    m = sum(m_bfs[:S]) + sum(m_sssp[:S])
    model, nproc, affinity = cpu_info()
    return {"value": round(m / t / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{S} steps (batch + BFS + SSSP) of the same workload after the bulk load and warm-up "
                      f"batches; the sequential C oracle pinned to one core",
            "seconds": round(t, 2), "matches_gpu": same,
            "cpu_model": model, "nproc": nproc, "affinity_cpus": affinity}


def synth_load(gr):
    from paper_2109_09527_amd import synth
    return synth.load_ops(gr)


if __name__ == "__main__":
    main()
