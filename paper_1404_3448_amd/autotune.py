"""Autotuner for the kernel plan of liblor.so.

Measures, on the current GPU, every value of each tuning knob and keeps the
fastest (coordinate descent in the order below), then writes the plan as
JSON keyed by the GPU architecture:

  digit_bits x radix_items_u32 : stable sort of 2^27 random 32-bit keys
  radix_items_u64              : stable sort of 2^26 random 58-bit keys
  merge_items                  : suffix array of a 64M-base noncoding-like text
  plcp_steps                   : LCP of the same text

then tunes a second plan for the batched entry point the same way (every
knob, starting from the plan above) on 512 pairs of the batched workload's
generator (pair totals log-uniform in [1e3, 1e6]), and times both plans
against the defaults on a 256M-base text (suffix array + LCP) and on the
batched pairs. A plan changes speed only; results are identical under every
plan.

    python -m paper_1404_3448_amd.autotune [--out DIR]   # writes plans/<arch>.json (or DIR/<arch>.json)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import lor, synth

PLAN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plans")


def arch_key() -> str:
    import torch
    name = getattr(torch.cuda.get_device_properties(0), "gcnArchName", "") or torch.cuda.get_device_name(0)
    return name.split(":")[0]


def plan_path(arch: str | None = None) -> str:
    return os.path.join(PLAN_DIR, f"{arch or arch_key()}.json")


def load_tuned_plan(apply: bool = True):
    """Read the tuned plan of this GPU (if any) and make it the process-wide plan."""
    try:
        with open(plan_path()) as f:
            doc = json.load(f)
    except OSError:
        return None
    if apply:
        lor.lor_plan_set(doc["plan"])
    return doc["plan"]


def load_batched_plan():
    """The plan tuned for the batched entry point on this GPU (None: use the process-wide plan)."""
    try:
        with open(plan_path()) as f:
            return json.load(f).get("batched_plan")
    except OSError:
        return None


def _time(fn, reps: int = 3) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def tune(log=print) -> dict:
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(0)
    best = lor.lor_plan_default().as_dict()
    meas = {}

    n32 = 1 << 27
    k32 = torch.from_numpy(rng.integers(0, 1 << 32, size=n32, dtype=np.uint64).astype(np.uint32).view(np.int32)).to(dev)
    v32 = torch.arange(n32, dtype=torch.int32, device=dev)
    kk, vv = torch.empty_like(k32), torch.empty_like(v32)
    ws32 = torch.empty(lor.lor_sort_pairs_workspace(n32, 4), dtype=torch.uint8, device=dev)

    def sort32():
        kk.copy_(k32)
        vv.copy_(v32)
        lor.lor_sort_pairs_u32(kk, vv, 0, 32, ws=ws32)

    for bits in (6, 7, 8):
        for items in (8, 12, 16, 24):
            lor.lor_plan_set(dict(best, digit_bits=bits, radix_items_u32=items))
            t = _time(sort32)
            meas[f"sort_u32 digit_bits={bits} items={items}"] = t
            log(f"sort u32 2^27: digit_bits={bits} items={items}: {1e3 * t:.2f} ms")
    key = min((k for k in meas if k.startswith("sort_u32")), key=meas.get)
    best["digit_bits"] = int(key.split("digit_bits=")[1].split()[0])
    best["radix_items_u32"] = int(key.split("items=")[1])
    del k32, v32, kk, vv, ws32

    n64 = 1 << 26
    k64 = torch.from_numpy((rng.integers(0, 1 << 58, size=n64, dtype=np.uint64)).view(np.int64)).to(dev)
    v64 = torch.arange(n64, dtype=torch.int32, device=dev)
    kk, vv = torch.empty_like(k64), torch.empty_like(v64)
    ws64 = torch.empty(lor.lor_sort_pairs_workspace(n64, 8), dtype=torch.uint8, device=dev)

    def sort64():
        kk.copy_(k64)
        vv.copy_(v64)
        lor.lor_sort_pairs_u64(kk, vv, 0, 58, ws=ws64)

    for items in (8, 12, 16):
        lor.lor_plan_set(dict(best, radix_items_u64=items))
        t = _time(sort64)
        meas[f"sort_u64 items={items}"] = t
        log(f"sort u64 2^26: items={items}: {1e3 * t:.2f} ms")
    best["radix_items_u64"] = int(min((k for k in meas if k.startswith("sort_u64")), key=meas.get).split("=")[1])
    del k64, v64, kk, vv, ws64

    w = synth.long_text(seed=3, num_seqs=4, seq_len=1 << 24, num_queries=1)
    seqs = torch.from_numpy(w.concat).to(dev)
    N = w.joined_length
    joined = torch.empty(N, dtype=torch.uint8, device=dev)
    sa = torch.empty(N, dtype=torch.int32, device=dev)
    lcp = torch.empty(N, dtype=torch.int32, device=dev)
    ws_sa = torch.empty(lor.lor_build_sa_workspace(int(w.offsets[-1]), 4), dtype=torch.uint8, device=dev)
    ws_lcp = torch.empty(lor.lor_build_lcp_workspace(N), dtype=torch.uint8, device=dev)
    for items in (4, 8, 12):
        lor.lor_plan_set(dict(best, merge_items=items))
        t = _time(lambda: lor.lor_build_sa(seqs, w.offsets, joined_out=joined, sa_out=sa, ws=ws_sa))
        meas[f"build_sa merge_items={items}"] = t
        log(f"suffix array 64M: merge_items={items}: {1e3 * t:.2f} ms")
    best["merge_items"] = int(min((k for k in meas if k.startswith("build_sa")), key=meas.get).split("=")[1])
    lor.lor_plan_set(best)
    lor.lor_build_sa(seqs, w.offsets, joined_out=joined, sa_out=sa, ws=ws_sa)
    for steps in (32, 64, 128, 256, 512):
        lor.lor_plan_set(dict(best, plcp_steps=steps))
        t = _time(lambda: lor.lor_build_lcp(joined, sa, lcp_out=lcp, ws=ws_lcp))
        meas[f"build_lcp plcp_steps={steps}"] = t
        log(f"LCP 64M: plcp_steps={steps}: {1e3 * t:.2f} ms")
    best["plcp_steps"] = int(min((k for k in meas if k.startswith("build_lcp")), key=meas.get).split("=")[1])
    lor.lor_plan_set(best)
    del seqs, joined, sa, lcp, ws_sa, ws_lcp

    # the batched entry point: every knob again, on the batched workload's pairs
    pairs = synth.batched_pairs(seed=40, num_pairs=512)
    bseqs = [x for p in pairs for x in p.seqs]
    boffs = np.concatenate([[0], np.cumsum([x.size for x in bseqs])]).astype(np.int64)
    bd = torch.from_numpy(np.concatenate(bseqs)).to(dev)
    bws = torch.empty(lor.lor_longest_overlap_batched_workspace(int(boffs[-1]), len(pairs)), dtype=torch.uint8,
                      device=dev)
    bout = torch.empty(len(pairs) * 32, dtype=torch.uint8, device=dev)
    log(f"batched tuning workload: {len(pairs)} pairs, {int(boffs[-1])} bases")

    def batched(plan):
        return _time(lambda: lor.lor_longest_overlap_batched(bd, boffs, out=bout, ws=bws, plan=plan))

    bbest = dict(best)
    knobs = [("digit_bits", (6, 7, 8)), ("radix_items_u32", (8, 12, 16, 24)), ("radix_items_u64", (8, 12, 16)),
             ("merge_items", (4, 8, 12)), ("plcp_steps", (32, 64, 128))]
    for knob, values in knobs:
        ts = {}
        for v in values:
            ts[v] = batched(dict(bbest, **{knob: v}))
            meas[f"batched {knob}={v}"] = ts[v]
            log(f"batched 512 pairs: {knob}={v}: {1e3 * ts[v]:.2f} ms")
        bbest[knob] = min(ts, key=ts.get)
    default = lor.lor_plan_default().as_dict()
    meas["check batched default plan"] = batched(default)
    meas["check batched batched plan"] = batched(bbest)
    del bd, bws, bout

    # both plans against the defaults on a larger text
    w = synth.long_text(seed=5, num_seqs=4, seq_len=1 << 26, num_queries=1)
    seqs = torch.from_numpy(w.concat).to(dev)
    N = w.joined_length
    joined = torch.empty(N, dtype=torch.uint8, device=dev)
    sa = torch.empty(N, dtype=torch.int32, device=dev)
    lcp = torch.empty(N, dtype=torch.int32, device=dev)
    ws_sa = torch.empty(lor.lor_build_sa_workspace(int(w.offsets[-1]), 4), dtype=torch.uint8, device=dev)
    ws_lcp = torch.empty(lor.lor_build_lcp_workspace(N), dtype=torch.uint8, device=dev)

    def sa_lcp():
        lor.lor_build_sa(seqs, w.offsets, joined_out=joined, sa_out=sa, ws=ws_sa)
        lor.lor_build_lcp(joined, sa, lcp_out=lcp, ws=ws_lcp)

    for name, plan in (("default", default), ("tuned", best)):
        lor.lor_plan_set(plan)
        meas[f"check sa+lcp 256M {name} plan"] = _time(sa_lcp, reps=2)
        log(f"SA + LCP 256M, {name} plan: {1e3 * meas[f'check sa+lcp 256M {name} plan']:.1f} ms")
    lor.lor_plan_set(best)
    return {"arch": arch_key(), "device": torch.cuda.get_device_name(0), "plan": best, "batched_plan": bbest,
            "measurements_ms": {k: round(1e3 * v, 3) for k, v in meas.items()},
            "command": "python -m paper_1404_3448_amd.autotune"}


def main():
    import argparse
    ap = argparse.ArgumentParser(description="tune the kernel plan of liblor.so on this GPU")
    ap.add_argument("--out", default=PLAN_DIR, help="directory for <arch>.json (default: the package's plans/)")
    args = ap.parse_args()
    doc = tune(log=lambda *a: print(*a, file=sys.stderr, flush=True))
    os.makedirs(args.out, exist_ok=True)
    path = os.path.join(args.out, f"{doc['arch']}.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print(json.dumps(doc["plan"]))
    print(f"wrote {path}", file=sys.stderr)


if __name__ == "__main__":
    main()
