"""Benchmark of the longest-overlap-region path on one MI355X.

One step = the whole path over one text already resident in HBM:
join -> DC3 suffix array -> LCP (+ ISA) -> sparse-table RMQ build ->
10M suffix-pair lcp queries -> longest overlap scan.

Default workload: 16 noncoding-like sequences of 67,108,864 bases (40% GC,
tandem repeats over ~10% of each), joined length N = 1,073,741,840, with
10,000,000 uniform (i, j) queries (seed 3). `value` is N / step time in
Msuffixes/s for the whole step; the SA+LCP-only rate is reported beside it.

After the timed steps:
* `end_to_end_with_h2d`: one step with the bases copied in from pinned host
  memory first (never `value`);
* `configs`: the 50k + 50k pair (latency, parity with the oracle's scan and
  its O(nm) DP, oracle times) and the 8M + 8M pair with 20 planted mutated
  segments (N / (t_SA + t_LCP), per-kernel rates, parity, rate with H2D);
* `ref_queries` and `ref_queries_sweep`: one reference against 65,536 query
  sequences, and against 512 ... 1,048,576 of them;
* `batched`: 4096 independent pairs (seed 4) through one batched call
  against a loop of the plain per-pair path, its HIP graph, a 64-pair batch
  eager against its graph, and the oracle looped over a sample of the pairs;
* `serving`: the continuous-batching loop under Poisson load (p50/p99);
* `cpu_baseline`: the CPU oracle on a bounded sample of the same text.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DC3 SA+LCP Msuffixes/s at 1G bases; batched pairs/s vs plain, bit-exact"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (num_seqs, seq_len, num_queries)
    "1g": (16, 1 << 26, 10_000_000),
    "8m": (2, 1 << 23, 1_000_000),
    "1m": (2, 1 << 20, 100_000),
}


def source_hash() -> str:
    from paper_1404_3448_amd.build import source_hash as h
    return h()


def committed_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs, or None
    when they were taken on other kernel sources (or not at all)."""
    path = os.path.join(ROOT, "profiles", "traffic_1g_path.json")
    try:
        with open(path) as f:
            doc = json.load(f)
    except OSError:
        return None
    k = doc.get("kernels", {}).get(kernel)
    if doc.get("source_sha256") != source_hash() or not k or not k.get("launches"):
        return None
    return round((k["read_bytes"] + k["write_bytes"]) / k["launches"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(seqs, seq_cut: int, nseq: int, threads: int) -> dict:
    """The CPU oracle (comparison-sort SA, direct LCP, overlap scan) on the
    first `nseq` sequences cut to `seq_cut` bases each."""
    import oracle

    sub = [s[:seq_cut] for s in seqs[:nseq]]
    offs = np.concatenate([[0], np.cumsum([s.size for s in sub])]).astype(np.int64)
    cat = np.concatenate(sub)
    t0 = time.perf_counter()
    joined = oracle.join(cat, offs)
    sa = oracle.suffix_array(joined, nthreads=threads)
    lcp = oracle.lcp(joined, sa, nthreads=threads)
    oracle.overlap(sa, lcp, offs)
    dt = time.perf_counter() - t0
    # one core, on a smaller sample of the same text
    sub1 = [s[: 1 << 22] for s in seqs[:2]]
    offs1 = np.concatenate([[0], np.cumsum([s.size for s in sub1])]).astype(np.int64)
    t1 = time.perf_counter()
    j1 = oracle.join(np.concatenate(sub1), offs1)
    sa1 = oracle.suffix_array(j1, nthreads=1)
    oracle.overlap(sa1, oracle.lcp(j1, sa1, nthreads=1), offs1)
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(joined.size / dt / 1e6, 3), "unit": "Msuffixes/s", "cores": threads, "kind": "oracle",
            "sample": f"first {nseq} sequences cut to {seq_cut} bases (N = {joined.size}); join + "
                      f"comparison-sort SA + direct LCP + overlap scan, {dt:.2f} s",
            "seconds": round(dt, 3),
            "single_core": {"value": round(j1.size / dt1 / 1e6, 3), "unit": "Msuffixes/s",
                            "sample": f"first 2 sequences cut to {1 << 22} bases (N = {j1.size}), {dt1:.2f} s"},
            "cpu_model": model, "nproc": os.cpu_count()}


def bench_batched(lor, synth, torch, reps: int = 3) -> dict:
    """4096 pairs (totals log-uniform in [1e3, 1e6], seed 4): one batched call
    versus a loop of the plain per-pair path, resident inputs, same results."""
    import ctypes

    from paper_1404_3448_amd import autotune
    bplan = autotune.load_batched_plan()      # tuned for the batched call (None: the process-wide plan)
    t0 = time.perf_counter()
    ws_pairs = synth.batched_pairs()
    seqs = [s for w in ws_pairs for s in w.seqs]
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    P = len(ws_pairs)
    total = int(offs[-1])
    log(f"batched workload: {P} pairs, {total} bases, generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    d = torch.from_numpy(np.concatenate(seqs)).to(dev)
    out = torch.empty(P * ctypes.sizeof(lor.lor_overlap), dtype=torch.uint8, device=dev)
    ws = torch.empty(lor.lor_longest_overlap_batched_workspace(total, P), dtype=torch.uint8, device=dev)
    lor.lor_longest_overlap_batched(d, offs, out=out, ws=ws, plan=bplan)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        lor.lor_longest_overlap_batched(d, offs, out=out, ws=ws, plan=bplan)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t) / reps
    batched = lor.records_to_tuples(out)
    del ws

    # the same call captured as a HIP graph and replayed (status() waits)
    side = torch.cuda.Stream()
    g = lor.lor_longest_overlap_batched_graph_create(d, offs, side, plan=bplan)
    side.synchronize()
    g.launch(side)
    g.status(side)
    t = time.perf_counter()
    for _ in range(reps):
        g.launch(side)
        g.status(side)
    graph_s = (time.perf_counter() - t) / reps
    graph_same = lor.records_to_tuples(g.out) == batched
    graph_levels = g.levels
    g.close()
    del g

    nmax = max(w.joined_length for w in ws_pairs)
    bmax = max(int(w.offsets[-1]) for w in ws_pairs)
    joined = torch.empty(nmax, dtype=torch.uint8, device=dev)
    sa = torch.empty(nmax, dtype=torch.int32, device=dev)
    lcp = torch.empty(nmax, dtype=torch.int32, device=dev)
    ws_sa = torch.empty(lor.lor_build_sa_workspace(bmax, 2), dtype=torch.uint8, device=dev)
    ws_lcp = torch.empty(lor.lor_build_lcp_workspace(nmax), dtype=torch.uint8, device=dev)
    ws_ov = torch.empty(lor.lor_longest_overlap_workspace(nmax, 2), dtype=torch.uint8, device=dev)
    plain = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for p, w in enumerate(ws_pairs):
        lo, hi = int(offs[2 * p]), int(offs[2 * p + 2])
        sub = w.offsets
        n = w.joined_length
        s_, j_ = lor.lor_build_sa(d[lo:hi], sub, joined_out=joined, sa_out=sa, ws=ws_sa)
        l_, _ = lor.lor_build_lcp(j_, s_, lcp_out=lcp, ws=ws_lcp)
        plain.append(lor.lor_longest_overlap(s_, l_, sub, ws=ws_ov))
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t
    return {"workload": f"{P} pairs, pair totals log-uniform in [1e3, 1e6], {total} bases (seed 4)",
            "pairs": P, "bases": total,
            "batched_ms": round(1e3 * batched_s, 3), "batched_pairs_per_s": round(P / batched_s, 1),
            "graph_ms": round(1e3 * graph_s, 3), "graph_pairs_per_s": round(P / graph_s, 1),
            "graph_dc3_levels": graph_levels, "graph_identical": graph_same,
            "plain_loop_ms": round(1e3 * plain_s, 3), "plain_loop_pairs_per_s": round(P / plain_s, 1),
            "speedup": round(plain_s / batched_s, 2), "identical_to_plain": batched == plain,
            "plan": bplan or "process-wide", "plan_source": "autotuned for the batched call" if bplan else "process-wide"}


def bench_ref_queries(lor, synth, torch, reps: int = 3, loop_sample: int = 256) -> dict:
    """One 4M-base reference against 65,536 queries (lengths log-uniform in
    [100, 2000], a third carrying a mutated reference segment; seed 6): one
    call over all queries versus the plain per-pair path on a sample."""
    t0 = time.perf_counter()
    w = synth.ref_queries()
    offs = w.offsets
    Q = len(w.seqs) - 1
    log(f"reference vs queries: {Q} queries, {int(offs[-1])} bases, generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    d = torch.from_numpy(w.concat).to(dev)
    out = torch.empty(Q * 32, dtype=torch.uint8, device=dev)
    ws = torch.empty(lor.lor_longest_overlap_ref_workspace(int(offs[-1]), Q), dtype=torch.uint8, device=dev)
    lor.lor_longest_overlap_ref(d, offs, out=out, ws=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        lor.lor_longest_overlap_ref(d, offs, out=out, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    recs = lor.records_to_tuples(out)
    del ws
    # the plain path, one (query, reference) pair at a time, on a sample
    ref = w.seqs[0]
    same = True
    t = time.perf_counter()
    for q in range(1, loop_sample + 1):
        query = w.seqs[q]
        po = np.array([0, query.size, query.size + ref.size], np.int64)
        pd = torch.from_numpy(np.concatenate([query, ref])).to(dev)
        ov = lor.longest_overlap_region(pd, po)["overlap"]
        same &= recs[q - 1][0] == ov[0] and (ov[0] == 0 or recs[q - 1][2] == ov[2])
    torch.cuda.synchronize()
    loop_s = (time.perf_counter() - t) / loop_sample
    return {"workload": f"reference of {ref.size} bases, {Q} queries of 100..2000 bases (log-uniform), "
                        f"{int(offs[-1])} bases in total (seed 6)",
            "queries": Q, "ms": round(1e3 * dt, 3), "queries_per_s": round(Q / dt, 1),
            "Mbases_per_s": round(int(offs[-1]) / dt / 1e6, 1),
            "plain_per_query_ms": round(1e3 * loop_s, 3), "speedup_vs_plain_loop": round(loop_s * Q / dt, 1),
            "plain_sample": loop_sample, "sample_identical_length_and_query_offset": bool(same)}


def bench_matrix(lor, torch, sa, lcp, offsets, num_seqs, N, ov, dev) -> dict:
    """All-pairs overlap matrix of the step's sequences, on its SA and LCP."""
    mout = torch.empty(num_seqs * num_seqs * 32, dtype=torch.uint8, device=dev)
    mws = torch.empty(lor.lor_overlap_matrix_workspace(N, num_seqs), dtype=torch.uint8, device=dev)
    lor.lor_overlap_matrix(sa, lcp, offsets, out=mout, ws=mws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    lor.lor_overlap_matrix(sa, lcp, offsets, out=mout, ws=mws)
    torch.cuda.synchronize()
    t = time.perf_counter() - t
    rec = lor.records_to_tuples(mout)
    L = [[rec[a * num_seqs + b][0] for b in range(num_seqs)] for a in range(num_seqs)]
    return {"sequences": num_seqs, "ms": round(1e3 * t, 3),
            "max_equals_longest_overlap": max(max(r) for r in L) == ov[0],
            "symmetric": all(L[a][b] == L[b][a] for a in range(num_seqs) for b in range(num_seqs)),
            "lengths": L}


def bench_rmq_compact(lor, torch, lcp, isa, qi, qj, qout, N, nq, stages, dev) -> dict:
    """The low-memory (block) table on the step's LCP, with the same queries."""
    ctab = torch.empty(lor.lor_rmq_compact_bytes(N) // 4, dtype=torch.int32, device=dev)
    cout = torch.empty(nq, dtype=torch.int32, device=dev)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    crmq = lor.lor_rmq_compact_build(lcp, table=ctab)
    lor.lor_rmq_query(crmq, lcp, isa, 1, qi, qj, min_out=cout)
    torch.cuda.synchronize()
    e0.record()
    crmq = lor.lor_rmq_compact_build(lcp, table=ctab)
    e1.record()
    lor.lor_rmq_query(crmq, lcp, isa, 1, qi, qj, min_out=cout)
    e2.record()
    torch.cuda.synchronize()
    return {"bytes": lor.lor_rmq_compact_bytes(N), "full_table_bytes": lor.lor_rmq_bytes(N),
            "build_ms": round(e0.elapsed_time(e1), 3), "queries_ms": round(e1.elapsed_time(e2), 3),
            "full_build_ms": stages["rmq_build"], "full_queries_ms": stages["queries"],
            "identical_to_full_table": bool(torch.equal(cout, qout))}


def _event_ms(torch, fn, reps: int) -> list:
    """Per-call device time of fn() on the current stream (HIP events), after one untimed call."""
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def bench_c1(lor, synth, torch) -> dict:
    """50k + 50k uniform bases with one exact 500-base copy (seed 1): latency
    of the whole path on resident input (join, SA, LCP, overlap), parity with
    the oracle's SA-scan overlap and its O(nm) DP, and the oracle times."""
    import oracle
    w = synth.tiny_pair(seed=1, n=50_000, planted_len=500)
    dev = torch.device("cuda:0")
    d = torch.from_numpy(w.concat).to(dev)
    N = w.joined_length
    joined = torch.empty(N, dtype=torch.uint8, device=dev)
    sa = torch.empty(N, dtype=torch.int32, device=dev)
    lcp = torch.empty(N, dtype=torch.int32, device=dev)
    ws_sa = torch.empty(lor.lor_build_sa_workspace(int(w.offsets[-1]), 2), dtype=torch.uint8, device=dev)
    ws_lcp = torch.empty(lor.lor_build_lcp_workspace(N), dtype=torch.uint8, device=dev)
    ws_ov = torch.empty(lor.lor_longest_overlap_workspace(N, 2), dtype=torch.uint8, device=dev)
    res = {}

    def path():
        lor.lor_build_sa(d, w.offsets, joined_out=joined, sa_out=sa, ws=ws_sa)
        lor.lor_build_lcp(joined, sa, lcp_out=lcp, ws=ws_lcp)
        res["ov"] = lor.lor_longest_overlap(sa, lcp, w.offsets, ws=ws_ov)   # synchronises

    path()
    lat = []
    for _ in range(20):
        torch.cuda.synchronize()
        t = time.perf_counter()
        path()
        lat.append(1e6 * (time.perf_counter() - t))
    ov = res["ov"]
    t = time.perf_counter()
    j = oracle.join(w.concat, w.offsets)
    so = oracle.suffix_array(j, nthreads=1)
    lo = oracle.lcp(j, so, nthreads=1)
    ov_o = oracle.overlap(so, lo, w.offsets)
    t_sa = time.perf_counter() - t
    t = time.perf_counter()
    dp = oracle.lcs_dp(w.seqs[0], w.seqs[1])
    t_dp = time.perf_counter() - t
    return {"workload": "50,000 + 50,000 uniform bases, one exact 500-base copy (seed 1)", "joined_length": N,
            "latency_us_p50": round(float(np.median(lat)), 1), "latency_us_min": round(float(min(lat)), 1),
            "overlap": list(ov), "equals_oracle_scan": ov == ov_o,
            "equals_oracle_dp": (ov[0], ov[2], ov[4]) == dp,
            "certified": oracle.certify(j, sa.cpu().numpy(), lcp.cpu().numpy()) == -1,
            "oracle_sa_lcp_scan_one_core_s": round(t_sa, 3), "oracle_dp_s": round(t_dp, 3)}


def bench_c2(lor, synth, torch, threads: int) -> dict:
    """8M + 8M noncoding-like bases with 20 planted mutated segments (seed 2):
    N / (t_SA + t_LCP), per-kernel rates, overlap parity with the oracle, and
    the rate with the bases copied in from pinned host memory first."""
    import oracle
    w = synth.noncoding_pair(seed=2)
    dev = torch.device("cuda:0")
    N = w.joined_length
    host = torch.from_numpy(w.concat).pin_memory()
    d = torch.empty_like(host, device=dev)
    d.copy_(host)
    joined = torch.empty(N, dtype=torch.uint8, device=dev)
    sa = torch.empty(N, dtype=torch.int32, device=dev)
    lcp = torch.empty(N, dtype=torch.int32, device=dev)
    ws_sa = torch.empty(lor.lor_build_sa_workspace(int(w.offsets[-1]), 2), dtype=torch.uint8, device=dev)
    ws_lcp = torch.empty(lor.lor_build_lcp_workspace(N), dtype=torch.uint8, device=dev)
    ws_ov = torch.empty(lor.lor_longest_overlap_workspace(N, 2), dtype=torch.uint8, device=dev)
    t_sa = _event_ms(torch, lambda: lor.lor_build_sa(d, w.offsets, joined_out=joined, sa_out=sa, ws=ws_sa), 5)
    t_lcp = _event_ms(torch, lambda: lor.lor_build_lcp(joined, sa, lcp_out=lcp, ws=ws_lcp), 5)
    t_h2d = _event_ms(torch, lambda: d.copy_(host, non_blocking=True), 5)
    ms = float(np.median(t_sa)) + float(np.median(t_lcp))
    lor.lor_timing_only(None)
    lor.lor_timing_reset()
    lor.lor_timing_enable(True)
    lor.lor_build_sa(d, w.offsets, joined_out=joined, sa_out=sa, ws=ws_sa)
    lor.lor_build_lcp(joined, sa, lcp_out=lcp, ws=ws_lcp)
    torch.cuda.synchronize()
    kern = lor.lor_timing_read()
    lor.lor_timing_enable(False)
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "alg_GBps": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else 0.0}
               for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])[:12]}
    ov = lor.lor_longest_overlap(sa, lcp, w.offsets, ws=ws_ov)
    t = time.perf_counter()
    j = oracle.join(w.concat, w.offsets)
    so = oracle.suffix_array(j, nthreads=threads)
    lo = oracle.lcp(j, so, nthreads=threads)
    ov_o = oracle.overlap(so, lo, w.offsets)
    t_o = time.perf_counter() - t
    same = bool(np.array_equal(sa.cpu().numpy(), so) and np.array_equal(lcp.cpu().numpy(), lo))
    h2d = float(np.median(t_h2d))
    return {"workload": "8,388,608 + 8,388,608 noncoding-like bases, 20 planted segments of 1k-10k bases with "
                        "1% mutations (seed 2)", "joined_length": N,
            "msuffixes_per_s": round(N / (ms * 1e-3) / 1e6, 1), "sa_ms": round(float(np.median(t_sa)), 3),
            "lcp_ms": round(float(np.median(t_lcp)), 3), "h2d_ms": round(h2d, 3),
            "msuffixes_per_s_with_h2d": round(N / ((ms + h2d) * 1e-3) / 1e6, 1),
            "kernels": kernels, "overlap": list(ov), "sa_lcp_equal_oracle": same, "overlap_equals_oracle": ov == ov_o,
            "oracle_s": round(t_o, 3), "oracle_threads": threads}


def bench_c4_oracle_loop(synth, sample: int = 48) -> dict:
    """The oracle looped over the first pairs of the 4096-pair batch (one
    core): SA by comparison sort, LCP, overlap scan, per pair."""
    import oracle
    pairs = synth.batched_pairs()[:sample]
    t = time.perf_counter()
    bases = 0
    for w in pairs:
        j = oracle.join(w.concat, w.offsets)
        so = oracle.suffix_array(j, nthreads=1)
        oracle.overlap(so, oracle.lcp(j, so, nthreads=1), w.offsets)
        bases += int(w.offsets[-1])
    dt = time.perf_counter() - t
    return {"pairs": sample, "bases": bases, "seconds": round(dt, 3), "pairs_per_s": round(sample / dt, 2),
            "Mbases_per_s": round(bases / dt / 1e6, 3), "cores": 1}


def bench_refq_sweep(lor, synth, torch, counts=(512, 4096, 32768, 262144, 1048576)) -> dict:
    """lor_longest_overlap_ref over growing numbers of query sequences (the
    NUMBER axis of Table V; Section V runs 512 and more queries per
    reference): the same 4M-base reference, the first Q queries of one
    generated list."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = synth.ref_queries(num_queries=max(counts))
    gen_s = time.perf_counter() - t0
    offs_all = w.offsets
    d = torch.from_numpy(w.concat).to(dev)
    out = {"reference_bases": int(w.seqs[0].size), "generated_s": round(gen_s, 1), "points": []}
    for Q in counts:
        offs = offs_all[: Q + 2]
        total = int(offs[-1])
        rec = torch.empty(Q * 32, dtype=torch.uint8, device=dev)
        ws = torch.empty(lor.lor_longest_overlap_ref_workspace(total, Q), dtype=torch.uint8, device=dev)
        sub = d[:total]
        ts = []
        for r in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            lor.lor_longest_overlap_ref(sub, offs, out=rec, ws=ws)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        dt = float(np.median(ts))
        out["points"].append({"queries": Q, "bases": total, "ms": round(1e3 * dt, 3),
                              "queries_per_s": round(Q / dt, 1), "Mbases_per_s": round(total / dt / 1e6, 1)})
        del ws, rec
        torch.cuda.empty_cache()
    return out


def bench_small_batch_graph(lor, synth, torch, pairs: int = 64, reps: int = 50) -> dict:
    """A small batch (64 pairs of 1k-10k bases in total, seed 7): the batched
    call eager against its captured HIP graph, where launch overhead matters."""
    ws_pairs = synth.batched_pairs(seed=7, num_pairs=pairs, lo=1e3, hi=1e4)
    seqs = [x for w in ws_pairs for x in w.seqs]
    offs = np.concatenate([[0], np.cumsum([x.size for x in seqs])]).astype(np.int64)
    dev = torch.device("cuda:0")
    d = torch.from_numpy(np.concatenate(seqs)).to(dev)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        out = torch.empty(pairs * 32, dtype=torch.uint8, device=dev)
        ws = torch.empty(lor.lor_longest_overlap_batched_workspace(int(offs[-1]), pairs), dtype=torch.uint8,
                         device=dev)
    side.wait_stream(torch.cuda.current_stream())
    lor.lor_longest_overlap_batched(d, offs, out=out, ws=ws, stream=side)
    eager = lor.records_to_tuples(out)
    t = time.perf_counter()
    for _ in range(reps):
        lor.lor_longest_overlap_batched(d, offs, out=out, ws=ws, stream=side)
    side.synchronize()
    eager_s = (time.perf_counter() - t) / reps
    g = lor.lor_longest_overlap_batched_graph_create(d, offs, side)
    g.launch(side)
    g.status(side)
    t = time.perf_counter()
    for _ in range(reps):          # one replay at a time, waited for (as the eager call waits)
        g.launch(side)
        g.status(side)
    graph_s = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):          # replays queued back to back
        g.launch(side)
    g.status(side)
    piped_s = (time.perf_counter() - t) / reps
    same = lor.records_to_tuples(g.out) == eager
    levels = g.levels
    g.close()
    return {"workload": f"{pairs} pairs, pair totals log-uniform in [1e3, 1e4], {int(offs[-1])} bases (seed 7)",
            "eager_ms": round(1e3 * eager_s, 3), "graph_ms": round(1e3 * graph_s, 3),
            "graph_queued_ms": round(1e3 * piped_s, 3), "graph_speedup": round(eager_s / graph_s, 2),
            "graph_dc3_levels": levels, "identical": bool(same)}


def bench_serving(seed: int = 5) -> dict:
    """Poisson requests (each sequence 1e4..4e6 bases, log-uniform; 30% keep
    state and send 10^4 follow-up queries after an exponential delay of mean
    50 ms) at 0.7x the closed-loop capacity, 200 GB HBM budget. Capacity is
    measured on a backlog of 96 requests, with continuous batching and, for
    comparison, with every request on the plain path."""
    from paper_1404_3448_amd import serve

    backlog = serve.make_requests(seed=seed + 100, count=96, qps=1e9)
    for r in backlog:
        r.arrival = 0.0
    from paper_1404_3448_amd import autotune
    runner = serve.GpuRunner(plan=autotune.load_batched_plan())
    warm = serve.make_requests(seed=seed + 200, count=16, qps=1e9)
    for r in warm:
        r.arrival = 0.0
    serve.Server(runner=runner, slots=4, batch_max=4).run(warm)   # streams and pinned staging, made once
    cap = serve.Server(runner=runner, slots=4).run(backlog)
    capacity = cap["result_pairs_per_s"]      # backlog over the time to its last pair result
    plain = serve.Server(runner=runner, slots=4, batching=False).run(
        serve.make_requests(seed=seed + 100, count=48, qps=1e9))
    qps = 0.7 * capacity
    reqs = serve.make_requests(seed=seed, count=400, qps=qps)
    stats = serve.Server(runner=runner, slots=4).run(reqs)
    stats.update({"capacity_pairs_per_s": capacity, "capacity_p50_ms": cap["p50_ms"],
                  "capacity_with_followup_waits_pairs_per_s": cap["pairs_per_s"],
                  "plain_path_capacity_pairs_per_s": plain["result_pairs_per_s"],
                  "capacity_vs_plain_path": round(capacity / plain["result_pairs_per_s"], 2),
                  "offered_qps": round(qps, 1),
                  "workload": "Poisson arrivals at 0.7x capacity; sequences log-uniform in [1e4, 4e6] bases; "
                              "30% keep state, 10^4 follow-up queries each (seed 5); continuous batching"})
    return stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="1g", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the overlap matrix, compact RMQ, radix ablation and reference-vs-queries runs")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 50k+50k and 8M+8M workloads, the query-count sweep and the oracle loops")
    ap.add_argument("--calibrate", action="store_true",
                    help="copy 1 GiB device-to-device first (reference for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; runs on more than one GPU are not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1404_3448_amd import autotune, lor, synth

    tuned = autotune.load_tuned_plan()          # the committed plan of this GPU, if any
    num_seqs, seq_len, nq = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    w = synth.long_text(seed=3, num_seqs=num_seqs, seq_len=seq_len, num_queries=nq)
    log(f"generated {w.name} in {time.perf_counter() - t0:.1f} s")
    offsets = w.offsets
    N = w.joined_length
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    seqs = torch.from_numpy(w.concat).to(dev)
    qi = torch.from_numpy(w.queries[0]).to(dev)
    qj = torch.from_numpy(w.queries[1]).to(dev)
    joined = torch.empty(N, dtype=torch.uint8, device=dev)
    sa = torch.empty(N, dtype=torch.int32, device=dev)
    lcp = torch.empty(N, dtype=torch.int32, device=dev)
    isa = torch.empty(N, dtype=torch.int32, device=dev)
    qout = torch.empty(nq, dtype=torch.int32, device=dev)
    ws_sa = torch.empty(lor.lor_build_sa_workspace(int(offsets[-1]), num_seqs), dtype=torch.uint8, device=dev)
    ws_lcp = torch.empty(lor.lor_build_lcp_workspace(N), dtype=torch.uint8, device=dev)
    ws_ov = torch.empty(lor.lor_longest_overlap_workspace(N, num_seqs), dtype=torch.uint8, device=dev)
    table = torch.empty(lor.lor_rmq_bytes(N) // 4, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    log(f"allocated {torch.cuda.memory_allocated() / 2**30:.1f} GiB on {torch.cuda.get_device_name(dev)}")

    if args.calibrate:
        # kernels of known HBM bytes for the memory counters: a 1 GiB
        # device-to-device copy (reads and writes 1 GiB), a 1 GiB fill (writes
        # only) and a sum over 1 GiB of int32 (reads only)
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        dst.fill_(3)
        torch.cuda.synchronize()
        total = int(dst.view(torch.int32).sum())
        torch.cuda.synchronize()
        log(f"calibration: copy, fill and sum over 1 GiB done ({total})")
        del src, dst

    names = ["sa", "lcp", "rmq_build", "queries", "overlap"]

    def step(ev=None):
        if ev:
            ev[0].record()
        lor.lor_build_sa(seqs, offsets, joined_out=joined, sa_out=sa, ws=ws_sa)
        if ev:
            ev[1].record()
        lor.lor_build_lcp(joined, sa, lcp_out=lcp, isa_out=isa, ws=ws_lcp)
        if ev:
            ev[2].record()
        rmq = lor.lor_rmq_build(lcp, table=table)
        if ev:
            ev[3].record()
        lor.lor_rmq_query(rmq, lcp, isa, 1, qi, qj, min_out=qout)
        if ev:
            ev[4].record()
        ov = lor.lor_longest_overlap(sa, lcp, offsets, ws=ws_ov)
        if ev:
            ev[5].record()
        return ov

    for i in range(args.warmup):
        t = time.perf_counter()
        ov = step()
        torch.cuda.synchronize()
        log(f"warmup {i}: {1e3 * (time.perf_counter() - t):.1f} ms, overlap {ov}")

    # Per-kernel breakdown: one more untimed step with events around every
    # launch. The timed steps then carry events only around the launches of
    # the dominant kernel, whose live average duration gives the roofline.
    kernels = {}
    dom_live = None
    if not args.no_kernel_timing:
        lor.lor_timing_only(None)
        lor.lor_timing_reset()
        lor.lor_timing_enable(True)
        step()
        torch.cuda.synchronize()
        kernels = lor.lor_timing_read()
        dom_live = max(kernels.items(), key=lambda kv: kv[1]["ms"])[0] if kernels else None
        log(f"kernel breakdown step done; timing {dom_live} live")
        lor.lor_timing_reset()
        lor.lor_timing_only(dom_live)
    stage_ms = {k: 0.0 for k in names}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        ov = step(ev)
        ev[5].synchronize()
        for k, name in enumerate(names):
            stage_ms[name] += ev[k].elapsed_time(ev[k + 1])
        log(f"step {i}: {ev[0].elapsed_time(ev[5]):.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    live = {}
    if not args.no_kernel_timing:
        live = lor.lor_timing_read()
        lor.lor_timing_enable(False)
        lor.lor_timing_only(None)

    # End to end with the bases copied in from pinned host memory first (never `value`).
    e2e = None
    if not args.no_configs:
        host = torch.from_numpy(w.concat).pin_memory()
        ts = []
        for _ in range(2):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            seqs.copy_(host, non_blocking=True)
            ev[1].record()
            step()
            ev[2].record()
            ev[2].synchronize()
            ts.append((ev[0].elapsed_time(ev[1]), ev[0].elapsed_time(ev[2])))
        h2d_ms, tot_ms = min(ts, key=lambda x: x[1])
        e2e = {"h2d_ms": round(h2d_ms, 3), "step_with_h2d_ms": round(tot_ms, 3),
               "msuffixes_per_s_with_h2d": round(N / (tot_ms * 1e-3) / 1e6, 3), "source": "pinned host memory"}
        del host
        log(f"end to end with H2D: {e2e}")

    ms_per_step = 1e3 * elapsed / args.steps
    value = N / (elapsed / args.steps) / 1e6
    stages = {k: round(v / args.steps, 3) for k, v in stage_ms.items()}
    sa_lcp_ms = stages["sa"] + stages["lcp"]

    roofline = None
    kern_out = {}
    for name, k in sorted(kernels.items(), key=lambda kv: -kv[1]["ms"]):   # one step's worth
        gbs = k["bytes"] / (k["ms"] * 1e-3) / 1e9 if k["ms"] > 0 else 0.0
        kern_out[name] = {"launches_per_step": k["launches"], "ms_per_step": round(k["ms"], 3),
                          "alg_GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
        # HBM bytes the counters measured for this kernel (1G workload, same sources) over the same time
        per_launch = committed_traffic(name) if args.workload == "1g" and k["ms"] > 0 else None
        if per_launch is not None:
            kern_out[name]["hbm_GBps"] = round(per_launch * k["launches"] / (k["ms"] * 1e-3) / 1e9, 1)
    if live.get(dom_live):
        dom_name, dom = dom_live, live[dom_live]   # events over the timed steps
        achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
        traffic = committed_traffic(dom_name) if args.workload == "1g" else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom_name,
                    "launch_ms_avg": round(dom["ms"] / dom["launches"], 4),
                    "alg_bytes_per_launch_avg": round(dom["bytes"] / dom["launches"])}

    matrix = rmq_compact = abl = refq = None
    del table
    torch.cuda.empty_cache()
    if not args.no_extras:
        matrix = bench_matrix(lor, torch, sa, lcp, offsets, num_seqs, N, ov, dev)
        log(f"overlap matrix: {num_seqs}x{num_seqs} in {matrix['ms']} ms")
        rmq_compact = bench_rmq_compact(lor, torch, lcp, isa, qi, qj, qout, N, nq, stages, dev)
        log(f"compact RMQ: {rmq_compact}")
    del ws_sa, ws_lcp, ws_ov, joined, sa, lcp, isa, qout, seqs, qi, qj
    torch.cuda.empty_cache()
    if not args.no_extras:
        from paper_1404_3448_amd import ablation
        log("radix ablation (digit width, size alignment) ...")
        abl = ablation.run()
        log(f"ablation: {abl}")
        log("reference vs queries ...")
        refq = bench_ref_queries(lor, synth, torch)
        log(f"reference vs queries: {refq}")

    configs = refq_sweep = None
    if not args.no_configs:
        threads = min(16, os.cpu_count() or 1)
        log("50k + 50k ...")
        configs = {"c1": bench_c1(lor, synth, torch)}
        log(f"c1: {configs['c1']}")
        log("8M + 8M ...")
        configs["c2"] = bench_c2(lor, synth, torch, threads)
        log(f"c2: {configs['c2']}")
        torch.cuda.empty_cache()
        log("reference vs queries, query-count sweep ...")
        refq_sweep = bench_refq_sweep(lor, synth, torch)
        log(f"refq sweep: {refq_sweep}")
        torch.cuda.empty_cache()

    batched = None
    if not args.no_batched:
        log("batched vs plain loop ...")
        batched = bench_batched(lor, synth, torch)
        log(f"batched: {batched}")
        torch.cuda.empty_cache()
        batched["small_batch_graph"] = bench_small_batch_graph(lor, synth, torch)
        log(f"small batch: {batched['small_batch_graph']}")
        if not args.no_cpu_baseline:
            batched["oracle_loop"] = bench_c4_oracle_loop(synth)
            log(f"oracle loop over pairs: {batched['oracle_loop']}")

    serving = None
    if not args.no_serving:
        log("serving ...")
        serving = bench_serving()
        log(f"serving: {serving}")

    cpu = None
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        cut = min(seq_len, 1 << 25)
        log("timing the CPU oracle sample ...")
        cpu = cpu_baseline(w.seqs, cut, min(8, num_seqs), threads)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Msuffixes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{num_seqs} x {seq_len}-base noncoding-like sequences (40% GC, tandem repeats), "
                               f"joined N = {N}; SA + LCP + ISA + sparse-table RMQ + {nq} suffix-pair queries + "
                               f"longest overlap",
                   "num_seqs": num_seqs, "seq_len": seq_len, "joined_length": N, "queries": nq, "seed": 3,
                   "plan": lor.lor_plan_get().as_dict(), "plan_source": "autotuned" if tuned else "default"},
        "sa_lcp_msuffixes_per_s": round(N / (sa_lcp_ms * 1e-3) / 1e6, 3),
        "queries_per_s": round(nq / (stages["queries"] * 1e-3), 1) if stages["queries"] > 0 else None,
        "stages_ms": stages,
        "overlap": list(ov),
        "roofline": roofline,
        "kernels": kern_out,
        "batched": batched,
        "serving": serving,
        "rmq_compact": rmq_compact,
        "overlap_matrix": matrix,
        "radix_ablation": abl,
        "ref_queries": refq,
        "ref_queries_sweep": refq_sweep,
        "configs": configs,
        "end_to_end_with_h2d": e2e,
        "cpu_baseline": cpu,
        "paper_context": {"claim": "more than 20x over a serial CPU run (abstract, Section I)",
                          "hardware": "Intel Core i3-3110M host, GeForce 610M",
                          "gpu_over_single_core_oracle": (round(value / cpu["single_core"]["value"], 1)
                                                          if cpu else None)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
