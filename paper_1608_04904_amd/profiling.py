"""Summaries of rocprofv3 runs of the benchmark.

Reads the SQLite databases that rocprofv3 writes (one kernel-trace run and
two counter runs, FETCH_SIZE and WRITE_SIZE) and the JSON line the benchmark
printed in the kernel-trace run, and writes

* a text table per kernel: launches, mean duration, HBM bytes fetched and
  written per launch (counter values scaled by the factor that makes a plain
  device copy of known size read and write exactly its size), the achieved
  HBM rate, and the algorithmic bytes per launch with the rate they imply;
* a JSON file of the same traffic figures keyed by the library's kernel
  names, stamped with a hash of the HIP sources so that a reader of the
  figures can tell whether the kernels changed since they were measured.

    python -m paper_1608_04904_amd.profiling --trace kt.db --fetch f.db \
        --write w.db --bench-log kt.log --calibrate-mib 512 \
        --title "..." --command "rocprofv3 ..." [--command ...] \
        --out-txt profiles/x_kernels.txt --out-json profiles/x_traffic.json
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3
import statistics

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def kernel_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of the HIP sources."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# library kernel (rocprof name without namespace and template arguments) ->
# the name of the timed phase that brackets it in the library's own events
PHASE = {"k_stream_bin": "stream_bin", "k_chain": "chain", "k_scan_blocks": "scan_blocks",
         "k_scan_final": "scan_final", "k_scatter": "scatter", "k_collide": "collide",
         "k_collide_big": "collide", "k_chunk_scan": "chunk_scan", "k_cand_write": "cand_write",
         "k_list": "list", "k_analysis": "analysis"}


def short_name(full: str) -> str:
    s = full.replace("void ", "")
    s = re.sub(r"^rmp::", "", s)
    return re.sub(r"\(.*$", "", s).strip()


def base_name(full: str) -> str:
    return re.sub(r"<.*$", "", short_name(full))


def durations(db: str) -> dict:
    con = sqlite3.connect(db)
    d = collections.defaultdict(list)
    for name, dur in con.execute("select name, duration from kernels"):
        d[short_name(name)].append(dur / 1e3)           # ns -> us
    return d


def counters(db: str, counter: str) -> dict:
    con = sqlite3.connect(db)
    d = collections.defaultdict(list)
    for name, val in con.execute("select kernel_name, value from counters_collection where counter_name=?",
                                 (counter,)):
        d[short_name(name)].append(val)
    return d


def calibration(vals: dict, mib: int) -> float:
    """Scale factor that makes the copy of `mib` MiB read (or write) `mib`
    MiB: the counters report KiB per dispatch; the copy is the largest
    dispatch of the runtime's copy kernel."""
    cp = [v for k, vs in vals.items() if "copyBuffer" in k for v in vs]
    if not cp:
        raise SystemExit("no device copy in the counter run (run the benchmark with --calibrate-copy)")
    return mib * 1024.0 / max(cp)


def bench_line(log: str) -> dict:
    line = None
    with open(log) as f:
        for ln in f:
            if ln.startswith("{"):
                line = ln
    if line is None:
        raise SystemExit(f"no JSON line in {log}")
    return json.loads(line)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--bench-log", required=True)
    ap.add_argument("--calibrate-mib", type=int, default=512)
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out-txt", required=True)
    ap.add_argument("--out-json", required=True)
    a = ap.parse_args()

    dur = durations(a.trace)
    fetch = counters(a.fetch, "FETCH_SIZE")
    write = counters(a.write, "WRITE_SIZE")
    sf, sw = calibration(fetch, a.calibrate_mib), calibration(write, a.calibrate_mib)
    bl = bench_line(a.bench_log)
    kev = bl.get("kernels", {})
    rows, js = [], {}
    for k in sorted(dur, key=lambda k: -sum(dur[k])):
        us = statistics.mean(dur[k])
        f = statistics.median(fetch[k]) * sf / 1024 if k in fetch else None     # MB (2^20 B)
        w = statistics.median(write[k]) * sw / 1024 if k in write else None
        ph = PHASE.get(base_name(k))
        algo = None
        if ph and ph in kev and base_name(k) != "k_collide_big":
            algo = kev[ph].get("algorithmic_MB")
        rows.append((k, len(dur[k]), us, f, w, algo))
        if ph and f is not None and base_name(k) != "k_collide_big":
            js[ph] = dict(kernel=k, fetch_MB=round(f, 4), write_MB=round(w, 4), avg_us=round(us, 2),
                          algorithmic_MB=algo)
    with open(a.out_txt, "w") as o:
        o.write(a.title.rstrip() + "\n\nCommands (from the repository root, TMPDIR=/tmp):\n")
        for c in a.command:
            o.write(f"  {c}\n")
        o.write(f"\nKernel durations: the kernel-trace run.  fetch/write: median per dispatch of\n"
                f"FETCH_SIZE and WRITE_SIZE from the two counter runs, scaled so that the plain\n"
                f"{a.calibrate_mib} MiB device copy reads and writes {a.calibrate_mib} MiB "
                f"(FETCH x{sf:.4f}, WRITE x{sw:.4f}).\nMB = 2^20 bytes; GB/s = 1e9 bytes/s.  "
                f"algo_MB: algorithmic bytes per launch as the benchmark states them.\n"
                f"HIP sources hash {kernel_source_hash()}\n\n")
        o.write(f"{'kernel':52s} {'calls':>5s} {'avg_us':>9s} {'fetch_MB':>10s} {'write_MB':>10s} "
                f"{'HBM_GB/s':>9s} {'algo_MB':>9s} {'algo_GB/s':>9s} {'traffic/algo':>12s}\n")
        for k, n, us, f, w, algo in rows:
            tot = (f or 0) + (w or 0)
            gbs = tot * 1048576 / (us * 1e-6) / 1e9 if f is not None else float("nan")
            agbs = algo * 1048576 / (us * 1e-6) / 1e9 if algo else float("nan")
            ratio = tot / algo if algo and f is not None else float("nan")
            o.write(f"{k[:52]:52s} {n:5d} {us:9.2f} {f if f is not None else float('nan'):10.3f} "
                    f"{w if w is not None else float('nan'):10.3f} {gbs:9.1f} "
                    f"{algo if algo else float('nan'):9.2f} {agbs:9.1f} {ratio:12.3f}\n")
        ev = {k: v.get("avg_ms") for k, v in kev.items()}
        o.write(f"\nHIP-event averages (ms) of the library's timed phases in the same run: {json.dumps(ev)}\n")
    with open(a.out_json, "w") as o:
        json.dump(dict(source_hash=kernel_source_hash(),
                       note=f"FETCH_SIZE x {sf:.4f} + WRITE_SIZE x {sw:.4f} per dispatch (median), "
                            f"MB = 2^20 B; commands in {os.path.basename(a.out_txt)}",
                       kernels=js), o, indent=1)


if __name__ == "__main__":
    main()
