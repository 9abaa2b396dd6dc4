"""Summaries of rocprofv3 results for the measurement record.

rocprofv3 writes an SQLite database per run.  Two helpers read it:

  * kernel_times(db): calls and average duration per kernel (kernel trace);
  * traffic(...): HBM bytes per step of the N-1 scan from two counter runs
    (FETCH_SIZE, then WRITE_SIZE, both reported in KiB per dispatch), each
    scaled by what the same counter reads for a plain device copy of known
    size, so that the figure is in bytes that actually crossed HBM.

Usage (after the counter runs; paths are the -d/-o of each rocprofv3 call):

  python -m paper_2501_17529_amd.profiling traffic \\
      --fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db \\
      --copy-bytes N --prec fp32 --source-hash H --out profiles/scan_medium_traffic.txt
"""
from __future__ import annotations

import argparse
import json
import sqlite3
from collections import defaultdict

SCAN_KERNELS = ("k_scan_max", "k_scan_win")


def _short(name: str) -> str:
    n = name.replace("dcflow::(anonymous namespace)::", "").replace("void ", "")
    return n.split("(")[0]


def counter_per_dispatch(db: str, counter: str):
    """{kernel name: [counter value per dispatch]} (values of one dispatch summed
    over the instances the profiler reports them for)."""
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, dispatch_id, sum(value) from counters_collection "
        "where counter_name = ? group by kernel_name, dispatch_id", (counter,)).fetchall()
    out = defaultdict(list)
    for name, _, v in rows:
        out[_short(name)].append(float(v))
    return dict(out)


def kernel_times(db: str):
    """[(kernel, calls, average ns)] from a kernel-trace database."""
    con = sqlite3.connect(db)
    tabs = [r[0] for r in con.execute("select name from sqlite_master where type in ('table','view')")]
    name = next(t for t in tabs if t == "kernels") if "kernels" in tabs else None
    if name is None:
        raise RuntimeError(f"no kernel table in {db}: {tabs}")
    rows = con.execute(f"select name, end - start from {name}").fetchall()
    acc = defaultdict(list)
    for n, d in rows:
        acc[_short(n)].append(d)
    return sorted(((k, len(v), sum(v) / len(v)) for k, v in acc.items()), key=lambda z: -z[1] * z[2])


def _copy_scale(db: str, counter: str, nbytes: int) -> float:
    """Bytes per counted KiB, from the run of `bench.py --copy-calibration`: its
    device-to-device copies (the runtime's copy kernel) are the largest
    dispatches of a kernel named *copy*; the median of those is used."""
    per = counter_per_dispatch(db, counter)
    vals = [v for k, vs in per.items() if "copy" in k.lower() for v in vs]
    if not vals:
        raise RuntimeError(f"no copy kernel with {counter} in {db}: {sorted(per)}")
    big = sorted(v for v in vals if v >= 0.5 * max(vals))
    kib = big[len(big) // 2]
    return nbytes / (kib * 1024.0)


def traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, copy_bytes, prec, source_hash):
    rs = _copy_scale(copy_fetch_db, "FETCH_SIZE", copy_bytes)
    ws = _copy_scale(copy_write_db, "WRITE_SIZE", copy_bytes)
    fetch = counter_per_dispatch(fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(write_db, "WRITE_SIZE")
    per_kernel = {}
    total = 0.0
    names = [k for k in sorted(set(fetch) | set(write)) if k.startswith(SCAN_KERNELS) and
             not (prec == "fp32" and "<float" not in k or prec == "fp64" and "<double" not in k)]
    # the winner pass comes in two forms (with and without the column-maximum
    # record); the step's is the one dispatched most (the other only in the bench's
    # agg_i section)
    wins = [k for k in names if k.startswith("k_scan_win")]
    if len(wins) > 1:
        step_win = max(wins, key=lambda k: len(fetch.get(k, [])))
        names = [k for k in names if not k.startswith("k_scan_win") or k == step_win]
    for k in names:
        fv, wv = fetch.get(k, [0.0]), write.get(k, [0.0])
        fb = sum(fv) / len(fv) * 1024.0 * rs
        wb = sum(wv) / len(wv) * 1024.0 * ws
        per_kernel[k] = {"fetch_bytes": fb, "write_bytes": wb}
        total += fb + wb
    return {"source_hash": source_hash, "prec": prec, "bytes_per_launch": total,
            "per_kernel": per_kernel, "read_scale": rs, "write_scale": ws,
            "copy_bytes": copy_bytes}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    for n in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--out", "--prec",
              "--source-hash"):
        t.add_argument(n, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    a = ap.parse_args()
    if a.cmd == "traffic":
        res = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.prec,
                      a.source_hash)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res))
    else:
        for name, calls, avg in kernel_times(a.db):
            print(f"| `{name}` | {calls} | {avg / 1000:.1f} |")


if __name__ == "__main__":
    main()
