"""Summaries of rocprofv3 output for the dg kernels.

DIR is a rocprofv3 output directory holding either a rocpd database
(*_results.db, the default output format) or CSV files.

  python -m paper_2109_09527_amd.rocprof_summary stats DIR
      per-kernel calls / total / average duration
  python -m paper_2109_09527_amd.rocprof_summary pmc DIR
      per-kernel mean of every collected counter per dispatch
  python -m paper_2109_09527_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR KERNEL COPY_KERNEL COPY_BYTES [SRC...]
      HBM bytes per dispatch of KERNEL from a FETCH_SIZE run and a WRITE_SIZE
      run, each scaled by what the same counter reads for a plain copy kernel
      (COPY_KERNEL, which reads and writes COPY_BYTES) in the same run.
      SRC files (the kernel's sources) are fingerprinted, so a reader can
      tell whether the kernel changed since.  Prints one JSON object.

Kernel names are matched by substring; the copy's dispatch is the largest
value among dispatches whose name contains COPY_KERNEL.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys
from collections import defaultdict


def _find(d, pattern):
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def _db(d):
    return _find(d, "*_results.db")


def _sql(path, q):
    import sqlite3
    con = sqlite3.connect(path)
    try:
        return con.execute(q).fetchall()
    finally:
        con.close()


def stats(d):
    """[(name, calls, total_ms, avg_us)] sorted by total time."""
    out = defaultdict(lambda: [0, 0.0])
    for path in _db(d):
        # kernel dispatch durations in ns
        for name, n, tot in _sql(path, "select name, count(*), sum(duration) from kernels group by name"):
            out[name][0] += n
            out[name][1] += tot
    for path in ([] if out else _find(d, "*kernel_stats.csv")):
        with open(path) as f:
            for r in csv.DictReader(f):
                out[r["Name"]][0] += int(r["Calls"])
                out[r["Name"]][1] += float(r["TotalDurationNs"])
    if not out:
        raise SystemExit(f"no kernel records under {d}")
    rows = [(k, n, tot / 1e6, tot / n / 1e3) for k, (n, tot) in out.items()]
    return sorted(rows, key=lambda r: -r[2])


def _per_dispatch(d, counter=None):
    """{(kernel, counter): [value per dispatch]}"""
    vals = defaultdict(list)
    for path in _db(d):
        q = "select kernel_name, counter_name, value from counters_collection"
        if counter:
            q += f" where counter_name = '{counter}'"
        for name, cn, v in _sql(path, q):
            vals[(name, cn)].append(float(v))
    for path in ([] if vals else _find(d, "*counter_collection.csv")):
        with open(path) as f:
            for r in csv.DictReader(f):
                if counter is None or r["Counter_Name"] == counter:
                    vals[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no counter records under {d}")
    return vals


def pmc(d):
    return {k: (len(v), sum(v) / len(v)) for k, v in _per_dispatch(d).items()}


def traffic(fetch_dir, write_dir, kernel, copy_kernel, copy_bytes):
    res = {"kernel": kernel, "copy_kernel": copy_kernel, "copy_bytes": copy_bytes}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        vals = _per_dispatch(d, counter)
        kv = [v for (name, _), xs in vals.items() if kernel in name for v in xs]
        cv = [v for (name, _), xs in vals.items() if copy_kernel in name for v in xs]
        if not kv or not cv:
            raise SystemExit(f"{counter}: no dispatch of {kernel!r} or {copy_kernel!r}")
        copy_kib = max(cv)
        factor = copy_bytes / (copy_kib * 1024.0)   # true bytes per counted byte
        mean_kib = sum(kv) / len(kv)
        res[counter] = {"dispatches": len(kv), "mean_kib": round(mean_kib, 1), "copy_kib": round(copy_kib, 1),
                        "factor": round(factor, 4), "bytes_per_dispatch": round(mean_kib * 1024.0 * factor)}
    res["bytes_per_dispatch"] = res["FETCH_SIZE"]["bytes_per_dispatch"] + res["WRITE_SIZE"]["bytes_per_dispatch"]
    return res


def sources_digest(paths):
    """sha256 over the named files' bytes, in the given order."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        rows = stats(argv[1])
        grand = sum(r[2] for r in rows)
        print(f"{'kernel':<72} {'calls':>7} {'total_ms':>10} {'avg_us':>10} {'pct':>6}")
        for name, calls, tot, avg in rows:
            print(f"{name[:72]:<72} {calls:>7} {tot:>10.3f} {avg:>10.2f} {100 * tot / grand:>6.2f}")
    elif len(argv) >= 2 and argv[0] == "pmc":
        for (name, counter), (n, mean) in sorted(pmc(argv[1]).items()):
            print(f"{name[:64]:<64} {counter:<20} {n:>6} {mean:>16.1f}")
    elif len(argv) >= 6 and argv[0] == "traffic":
        res = traffic(argv[1], argv[2], argv[3], argv[4], int(argv[5]))
        if len(argv) > 6:
            res["sources"] = argv[6:]
            res["sources_sha256"] = sources_digest(argv[6:])
        print(json.dumps(res))
    else:
        print(__doc__, file=sys.stderr)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
