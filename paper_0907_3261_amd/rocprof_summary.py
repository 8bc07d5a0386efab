"""Summaries of rocprofv3 result databases for the wdsolve kernels.

    python -m paper_0907_3261_amd.rocprof_summary trace  RESULTS.db
    python -m paper_0907_3261_amd.rocprof_summary counters FETCH.db WRITE.db \
        --copy-bytes B --out traffic.json --src-hash H

``trace`` prints calls and average / min / max duration per kernel.
``counters`` prints FETCH_SIZE and WRITE_SIZE (KiB per dispatch) per kernel
and converts them to bytes per launch, each scaled by the ratio between the
known size of a plain copy (``--copy-bytes`` read and as many written; the
copy kernel is the one whose name contains ``copyBuffer``) and what the same
counter reports for it.
"""

from __future__ import annotations

import argparse
import json
import re
import sqlite3


def _short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("wd::", "")
    n = re.sub(r"\(.*\)$", "", n)
    return n


def trace(db: str):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    out = []
    for name, n, avg, mn, mx, tot in rows:
        out.append(dict(kernel=_short(name), calls=n, avg_us=avg / 1e3, min_us=mn / 1e3, max_us=mx / 1e3,
                        total_ms=tot / 1e6))
    return out


def counters(db: str):
    con = sqlite3.connect(db)
    rows = con.execute(
        "select kernel_name, counter_name, avg(value), count(*) from counters_collection "
        "group by kernel_name, counter_name").fetchall()
    return [dict(kernel=_short(k), counter=c, avg=v, n=n) for k, c, v, n in rows]


def main():
    p = argparse.ArgumentParser()
    p.add_argument("mode", choices=["trace", "counters"])
    p.add_argument("db", nargs="+")
    p.add_argument("--copy-bytes", type=float, default=None)
    p.add_argument("--out", default=None)
    p.add_argument("--src-hash", default=None)
    a = p.parse_args()
    if a.mode == "trace":
        print(f"{'calls':>6} {'avg_us':>11} {'min_us':>11} {'max_us':>11} {'total_ms':>10}  kernel")
        for r in trace(a.db[0]):
            print(f"{r['calls']:6d} {r['avg_us']:11.1f} {r['min_us']:11.1f} {r['max_us']:11.1f} "
                  f"{r['total_ms']:10.2f}  {r['kernel']}")
        return
    table = {}
    for db in a.db:
        for r in counters(db):
            table.setdefault(r["kernel"], {})[r["counter"]] = r["avg"]
    scale = {}
    copy = [k for k in table if "copyBuffer" in k]
    if a.copy_bytes and copy:
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            v = table[copy[0]].get(ctr)
            if v:
                scale[ctr] = a.copy_bytes / (v * 1024.0)
    print(f"copy calibration (bytes per reported KiB / 1024): {scale}")
    res = {}
    for k, d in table.items():
        f = d.get("FETCH_SIZE")
        w = d.get("WRITE_SIZE")
        line = f"{k}: FETCH_SIZE {f} KiB, WRITE_SIZE {w} KiB"
        if f is not None and w is not None and scale:
            b = f * 1024.0 * scale.get("FETCH_SIZE", 1.0) + w * 1024.0 * scale.get("WRITE_SIZE", 1.0)
            line += f" -> {b / 1e9:.3f} GB per launch (scaled)"
            res[k] = b
        print(line)
    if a.out:
        json.dump(dict(src_hash=a.src_hash, scale=scale, bytes_per_launch=res), open(a.out, "w"), indent=1)


if __name__ == "__main__":
    main()
