"""Summaries of rocprofv3 result databases for the wdsolve kernels.

    python -m paper_0907_3261_amd.rocprof_summary trace  RESULTS.db
    python -m paper_0907_3261_amd.rocprof_summary counters FETCH.db WRITE.db \
        --copy-bytes B --out traffic.json --src-hash H
    python -m paper_0907_3261_amd.rocprof_summary pipes P1.db P2.db P3.db

``trace`` prints calls and average / min / max duration per kernel.
``pipes`` prints, per kernel, where the memory pipeline of a CU spends its
time, from the counter passes TA_TA_BUSY_sum, TD_TD_BUSY_sum, TD_TC_STALL_sum,
TCP_TCC_READ_REQ_sum, TCP_TCC_READ_REQ_LATENCY_sum, SQ_ACTIVE_INST_VALU,
TCC_EA0_RDREQ_sum, TCC_EA0_RDREQ_128B_sum, TCC_HIT_sum with GRBM_GUI_ACTIVE
(summed over the 8 XCDs, so divided by 8 for the kernel's cycles): the
fraction of cycles the texture address (TA) and data (TD) units are busy,
the fraction TD waits for the L1 (TC), the L1 -> L2 read requests and
their average latency, the requests in flight per CU that this implies
(requests x latency / cycles / CUs), the L2 hit rate, the 128-byte reads
the L2 sends to the fabric (MALL or HBM) per launch, and the VALU-busy
fraction.
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


def pipes(dbs, cus: int = 256, xcds: int = 8):
    table = {}
    for db in dbs:
        for r in counters(db):
            table.setdefault(r["kernel"], {})[r["counter"]] = r["avg"]
    print(f"{'kernel':44s} {'TA':>5} {'TD':>5} {'TDwait':>6} {'L1req':>9} {'lat':>5} {'inflt/CU':>8} "
          f"{'L2hit':>6} {'fabricGB':>8} {'VALU':>5}")
    for k, d in table.items():
        need = ("GRBM_GUI_ACTIVE", "TA_TA_BUSY_sum", "TCP_TCC_READ_REQ_sum")
        if not all(n in d for n in need) or not d["TCP_TCC_READ_REQ_sum"]:
            continue
        cyc = d["GRBM_GUI_ACTIVE"] / xcds
        req = d["TCP_TCC_READ_REQ_sum"]
        lat = d.get("TCP_TCC_READ_REQ_LATENCY_sum", float("nan")) / req
        ea = d.get("TCC_EA0_RDREQ_sum", float("nan"))
        hit = d.get("TCC_HIT_sum", float("nan"))
        fab = d.get("TCC_EA0_RDREQ_128B_sum", float("nan")) * 128 / 1e9
        valu = d.get("SQ_ACTIVE_INST_VALU", float("nan")) / cus / cyc
        print(f"{k[:44]:44s} {d['TA_TA_BUSY_sum'] / cus / cyc:5.2f} {d.get('TD_TD_BUSY_sum', 0) / cus / cyc:5.2f} "
              f"{d.get('TD_TC_STALL_sum', 0) / cus / cyc:6.2f} {req:9.3g} {lat:5.0f} {req * lat / cyc / cus:8.1f} "
              f"{hit / (hit + ea):6.2f} {fab:8.2f} {valu:5.2f}")


def main():
    p = argparse.ArgumentParser()
    p.add_argument("mode", choices=["trace", "counters", "pipes"])
    p.add_argument("db", nargs="+")
    p.add_argument("--copy-bytes", type=float, default=None)
    p.add_argument("--out", default=None)
    p.add_argument("--src-hash", default=None)
    a = p.parse_args()
    if a.mode == "pipes":
        pipes(a.db)
        return
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
    if a.copy_bytes:
        # calibrate on the largest device copy of the run (the copy of copy_bytes; other, smaller
        # copies of the same kernel would dilute an average)
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            best = None
            for db in a.db:
                con = sqlite3.connect(db)
                r = con.execute("select max(value) from counters_collection where counter_name = ? and "
                                "kernel_name like '%copyBuffer%'", (ctr,)).fetchone()
                if r and r[0]:
                    best = r[0] if best is None else max(best, r[0])
            if best:
                scale[ctr] = a.copy_bytes / (best * 1024.0)
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
