"""Summaries of rocprofv3 output for the profiles/ notes (text only).

    python -m paper_1404_3448_amd.profsum stats KERNEL_STATS_CSV [--top N]
        per-kernel calls, total, average and share of kernel time (markdown)
    python -m paper_1404_3448_amd.profsum trace KERNEL_TRACE_CSV
        GPU busy time (union of kernel intervals) over the traced span, the
        time two or more kernels ran at once, and the streams that launched them
        (--split-gap-ms G: per phase, phases being separated by idle gaps > G ms)
    python -m paper_1404_3448_amd.profsum counters DIR [DIR ...] --kernels K1,K2,...
        every counter of the counter runs under the directories, summed over
        the dispatches of each named kernel (markdown)
    python -m paper_1404_3448_amd.profsum traffic FETCH_DIR WRITE_DIR --out JSON
        HBM bytes per kernel from a FETCH_SIZE and a WRITE_SIZE counter run
        (KiB per dispatch), scaled by what the same counters read for kernels
        of known bytes in the same run (`bench.py --calibrate`). FETCH_SIZE
        prices every read request at 64 bytes on this part (its 128-byte term,
        TCC_BUBBLE, reads 0), while requests are 64 or 128 bytes: the 1 GiB
        device-to-device copy (128-byte requests) reads 2x its FETCH_SIZE and
        the sum over 1 GiB (64-byte requests) 1x. read_bytes is therefore the
        upper bound (copy factor; streaming kernels issue 128-byte requests)
        and read_bytes_lo the lower bound (sum factor). WRITE_SIZE is scaled
        by the 1 GiB fill. The JSON carries the hash of the kernel sources it
        was taken on.

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


def trace(path: str, split_gap_ms: float = 0.0) -> str:
    rows = _rows(path)
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Stream_Id", r.get("Queue_Id")))
                for r in rows)
    if not iv:
        return "no kernels"
    if split_gap_ms > 0:   # phases: runs of kernels separated by idle gaps longer than split_gap_ms
        phases, cur, end = [], [iv[0]], iv[0][1]
        for x in iv[1:]:
            if x[0] - end > split_gap_ms * 1e6:
                phases.append(cur)
                cur = []
            cur.append(x)
            end = max(end, x[1])
        phases.append(cur)
        return "\n".join(f"phase {i}: " + _busy(p) for i, p in enumerate(phases))
    return _busy(iv)


def _busy(iv: list) -> str:
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
    sum_f, fill_w = first(fetch, is_sum), first(write, is_fill)
    if not (cf and cw and sum_f and fill_w):
        raise SystemExit("the 1 GiB copy, sum and fill of bench.py --calibrate are missing from the counter runs")
    ff, ff_lo, wf = GIB / cf, GIB / sum_f, GIB / fill_w
    cal = {"bytes": GIB, "copy_fetch_kib": cf / 1024, "copy_write_kib": cw / 1024, "sum_fetch_kib": sum_f / 1024,
           "fill_write_kib": fill_w / 1024, "fetch_factor": ff, "fetch_factor_lo": ff_lo, "write_factor": wf}
    kernels = {}
    for recs, keys, facs in ((fetch, ("read_bytes", "read_bytes_lo"), (ff, ff_lo)), (write, ("write_bytes",), (wf,))):
        seen = {}
        for _, name, b in recs:
            if "lor::" not in name:
                continue
            k = short(name)
            d = kernels.setdefault(k, {"launches": 0, "read_bytes": 0.0, "read_bytes_lo": 0.0, "write_bytes": 0.0})
            for key, fac in zip(keys, facs):
                d[key] += b * fac
            seen[k] = seen.get(k, 0) + 1
        for k, c in seen.items():
            kernels[k]["launches"] = max(kernels[k]["launches"], c)
    return {"calibration": cal, "source_sha256": source_sha256,
            "kernels": dict(sorted(kernels.items(), key=lambda x: -(x[1]["read_bytes"] + x[1]["write_bytes"])))}


def counters(dirs: list, kernels: list) -> str:
    sums = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in _rows(f):
                k = short(r["Kernel_Name"])
                if k in kernels:
                    key = (r["Counter_Name"], k)
                    sums[key] = sums.get(key, 0.0) + float(r["Counter_Value"])
    names = sorted({c for c, _ in sums})
    out = ["| counter | " + " | ".join(kernels) + " |", "|---|" + "---:|" * len(kernels)]
    for c in names:
        out.append(f"| {c} | " + " | ".join(f"{sums.get((c, k), 0.0):.3g}" for k in kernels) + " |")
    return "\n".join(out)


def traffic_table(doc: dict, top: int = 20) -> str:
    out = ["| kernel | launches | read GB (64 B .. 128 B requests) | write GB | bytes/launch (upper) |",
           "|---|---:|---:|---:|---:|"]
    for k, d in list(doc["kernels"].items())[:top]:
        per = (d["read_bytes"] + d["write_bytes"]) / max(d["launches"], 1)
        out.append(f"| {k} | {d['launches']} | {d['read_bytes_lo'] / 1e9:.1f} .. {d['read_bytes'] / 1e9:.1f} | "
                   f"{d['write_bytes'] / 1e9:.1f} | {per / 1e9:.3f} G |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=25)
    a = sub.add_parser("trace")
    a.add_argument("csv")
    a.add_argument("--split-gap-ms", type=float, default=0.0,
                   help="report phases separated by idle gaps longer than this")
    a = sub.add_parser("counters")
    a.add_argument("dirs", nargs="+")
    a.add_argument("--kernels", required=True)
    a = sub.add_parser("traffic")
    a.add_argument("fetch_dir")
    a.add_argument("write_dir")
    a.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.csv, args.top))
    elif args.cmd == "trace":
        print(trace(args.csv, args.split_gap_ms))
    elif args.cmd == "counters":
        print(counters(args.dirs, args.kernels.split(",")))
    else:
        from .build import source_hash
        doc = traffic(args.fetch_dir, args.write_dir, source_hash())
        with open(args.out, "w") as f:
            json.dump(doc, f, indent=1)
        print(json.dumps(doc["calibration"]), file=sys.stderr)
        print(traffic_table(doc))


if __name__ == "__main__":
    main()
