"""Summaries of rocprofv3 output for the profiles/ notes (text only).

    python -m paper_1404_3448_amd.profsum stats KERNEL_STATS_CSV [--top N]
        per-kernel calls, total, average and share of kernel time (markdown)
    python -m paper_1404_3448_amd.profsum trace KERNEL_TRACE_CSV
        GPU busy time (union of kernel intervals) over the traced span, the
        time two or more kernels ran at once, and the streams that launched them
    python -m paper_1404_3448_amd.profsum traffic FETCH_DIR WRITE_DIR --out JSON
        HBM bytes per kernel from a FETCH_SIZE and a WRITE_SIZE counter run
        (KiB per dispatch), each scaled by what the same counter reads for the
        1 GiB device-to-device copy of `bench.py --calibrate`; the fill
        (write-only) and sum (read-only) kernels of the same run are reported
        beside it as a check of the factors. The JSON carries the hash of the
        kernel sources it was taken on.

Kernel names are shortened to the function name (namespace, arguments and
template arguments dropped).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import sys

GIB = 1 << 30


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*", "", name)
    name = re.sub(r"<.*", "", name)
    return name.split("::")[-1].strip()


def _rows(path: str) -> list:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats(path: str, top: int = 25) -> str:
    rows = _rows(path)
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    merged = {}
    for r in rows:
        k = short(r["Name"])
        c, t = merged.get(k, (0, 0.0))
        merged[k] = (c + int(r["Calls"]), t + float(r["TotalDurationNs"]))
    out = ["| kernel | calls | total ms | avg ms | % |", "|---|---:|---:|---:|---:|"]
    for k, (c, t) in sorted(merged.items(), key=lambda x: -x[1][1])[:top]:
        out.append(f"| {k} | {c} | {t / 1e6:.2f} | {t / 1e6 / c:.4f} | {100 * t / tot:.1f} |")
    out.append(f"\nAll kernels: {tot / 1e6:.1f} ms.")
    return "\n".join(out)


def trace(path: str) -> str:
    rows = _rows(path)
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Stream_Id", r.get("Queue_Id")))
                for r in rows)
    if not iv:
        return "no kernels"
    ev = []
    for s, e, _ in iv:
        ev += [(s, 1), (e, -1)]
    ev.sort()
    busy = over = 0
    cur = 0
    last = ev[0][0]
    for t, d in ev:
        if cur >= 1:
            busy += t - last
        if cur >= 2:
            over += t - last
        cur += d
        last = t
    span = max(e for _, e, _ in iv) - iv[0][0]
    streams = len(set(x[2] for x in iv))
    return (f"{len(iv)} kernels from {streams} streams over {span / 1e6:.1f} ms; GPU busy (some kernel running) "
            f"{busy / 1e6:.1f} ms ({100 * busy / span:.0f}%), idle {(span - busy) / 1e6:.1f} ms; two or more kernels "
            f"at once {over / 1e6:.1f} ms ({100 * over / max(busy, 1):.0f}% of the busy time)")


def _counter(dirpath: str, counter: str) -> list:
    files = glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {dirpath}")
    out = []
    for f in files:
        for r in _rows(f):
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
    out.sort()
    return out


def traffic(fetch_dir: str, write_dir: str, source_sha256: str) -> dict:
    fetch = _counter(fetch_dir, "FETCH_SIZE")
    write = _counter(write_dir, "WRITE_SIZE")

    def first(recs, pred):
        return next((b for _, name, b in recs if pred(name)), None)

    is_copy = lambda n: "copyBuffer" in n
    is_fill = lambda n: "Fill" in n
    is_sum = lambda n: "reduce_kernel" in n
    cf, cw = first(fetch, is_copy), first(write, is_copy)
    if not cf or not cw:
        raise SystemExit("the 1 GiB copy of bench.py --calibrate is missing from the counter runs")
    ff, wf = GIB / cf, GIB / cw
    cal = {"copy_bytes": GIB, "fetch_kib": cf / 1024, "write_kib": cw / 1024, "fetch_factor": ff,
           "write_factor": wf}
    fill_w, sum_f = first(write, is_fill), first(fetch, is_sum)
    if fill_w:
        cal["fill_1gib_write_bytes_scaled"] = fill_w * wf
    if sum_f:
        cal["sum_1gib_fetch_bytes_scaled"] = sum_f * ff
    kernels = {}
    for recs, key, fac in ((fetch, "read_bytes", ff), (write, "write_bytes", wf)):
        seen = {}
        for _, name, b in recs:
            if not name.startswith("lor::"):
                continue
            k = short(name)
            d = kernels.setdefault(k, {"launches": 0, "read_bytes": 0.0, "write_bytes": 0.0})
            d[key] += b * fac
            seen[k] = seen.get(k, 0) + 1
        for k, c in seen.items():
            kernels[k]["launches"] = max(kernels[k]["launches"], c)
    return {"calibration": cal, "source_sha256": source_sha256,
            "kernels": dict(sorted(kernels.items(), key=lambda x: -(x[1]["read_bytes"] + x[1]["write_bytes"])))}


def traffic_table(doc: dict, top: int = 20) -> str:
    out = ["| kernel | launches | read GB | write GB | bytes/launch |", "|---|---:|---:|---:|---:|"]
    for k, d in list(doc["kernels"].items())[:top]:
        per = (d["read_bytes"] + d["write_bytes"]) / max(d["launches"], 1)
        out.append(f"| {k} | {d['launches']} | {d['read_bytes'] / 1e9:.1f} | {d['write_bytes'] / 1e9:.1f} | "
                   f"{per / 1e9:.3f} G |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=25)
    a = sub.add_parser("trace")
    a.add_argument("csv")
    a = sub.add_parser("traffic")
    a.add_argument("fetch_dir")
    a.add_argument("write_dir")
    a.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.csv, args.top))
    elif args.cmd == "trace":
        print(trace(args.csv))
    else:
        from .build import source_hash
        doc = traffic(args.fetch_dir, args.write_dir, source_hash())
        with open(args.out, "w") as f:
            json.dump(doc, f, indent=1)
        print(json.dumps(doc["calibration"]), file=sys.stderr)
        print(traffic_table(doc))


if __name__ == "__main__":
    main()
