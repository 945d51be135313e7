"""Serving loop for longest-overlap requests on one GPU (continuous batching).

Requests (a pair of DNA sequences, an arrival time, and optionally a batch of
follow-up suffix-pair lcp queries) arrive over time. The loop

* queues every arrival; whenever a worker slot is free it takes the queue's
  oldest requests (up to `batch_max` pairs and `batch_bases` bases, and what
  the HBM budget still admits) as one batch, so requests that arrive while
  others are on the GPU join the next batch as soon as a slot and memory
  free up, and batches on different slots overlap on the device;
* runs each batch through the batched entry point (one DC3 over all its
  pairs), on the worker's own HIP stream, with the bases staged through a
  pinned host buffer; when a request keeps state, the batch also returns its
  LCP and ISA, and the request's slices of them (its own LCP and ISA) stay
  resident with a compact block sparse table (about 8.4 bytes per base) until
  its follow-up query batch has been answered;
* charges every batch the exact bytes the library's size queries give
  (workspace, inputs, outputs, and the resident state of its keep-state
  requests) against the budget, and counts the times admission had to wait
  for memory;
* records arrival-to-result latency per request and per follow-up batch;
* keeps serving when a call fails (for instance a base outside 0..3): a
  failed batch of several requests is retried one request at a time, and
  only a request that fails alone is marked failed (its error kept).

With batching off every request runs alone on the plain path (SA, LCP,
overlap scan). All GPU work goes through the C-ABI (paper_1404_3448_amd.lor);
nothing here computes on the CPU besides bookkeeping.
"""
from __future__ import annotations

import ctypes
import heapq
import queue
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import lor


@dataclass
class Request:
    rid: int
    a: np.ndarray
    b: np.ndarray
    arrival: float                    # seconds after the start of the run
    keep: bool = False                # keep state for follow-up queries
    followup: tuple | None = None     # (qi, qj) int32 joined positions
    followup_delay: float = 0.0       # seconds after the result
    # filled in by the server
    result: tuple | None = None
    t_result: float | None = None
    followup_result: np.ndarray | None = None
    t_followup: float | None = None
    t_followup_arrival: float | None = None
    batched: bool = False
    rejected: bool = False
    error: str | None = None          # why the request (or its follow-up batch) failed

    @property
    def bases(self) -> int:
        return int(self.a.size + self.b.size)

    @property
    def offsets(self) -> np.ndarray:
        return np.array([0, self.a.size, self.a.size + self.b.size], dtype=np.int64)


def plain_bytes(total_bases: int, keep: bool) -> int:
    """Device bytes of one plain-path request: inputs, outputs and the largest
    workspace (the three calls run one after another and share it)."""
    n = total_bases + 2
    ws = max(lor.lor_build_sa_workspace(total_bases, 2), lor.lor_build_lcp_workspace(n),
             lor.lor_longest_overlap_workspace(n, 2))
    b = total_bases + n + 4 * n * 2 + ws          # seqs, joined, sa, lcp, workspace
    if keep:
        b += 4 * n + lor.lor_rmq_compact_bytes(n)   # isa + compact sparse table stay resident
    return int(b)


def resident_bytes(total_bases: int) -> int:
    """Bytes that stay after a keep-state request: LCP, ISA and the compact
    (block) sparse table."""
    n = total_bases + 2
    return int(4 * n * 2 + lor.lor_rmq_compact_bytes(n))


def batch_bytes(total_bases: int, pairs: int, keep: bool = False) -> int:
    """Device bytes of one batched call while it runs: bases, workspace and
    records, plus the whole batch's LCP and ISA when a request keeps state."""
    b = total_bases + lor.lor_longest_overlap_batched_workspace(total_bases, pairs) + pairs * ctypes.sizeof(
        lor.lor_overlap)
    if keep:
        b += 8 * (total_bases + 2 * pairs)
    return int(b)


class GpuRunner:
    """Device work of the serving loop. Every call takes a worker context (a
    HIP stream of default priority and a pinned staging buffer) from a pool
    that outlives the calls, so streams and pinned memory are made once."""

    def __init__(self, device: str = "cuda:0", plan=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.plan = plan              # plan of the batched calls (None: the process-wide plan)
        self._pool = queue.SimpleQueue()
        lor.lib()

    def _take(self) -> dict:
        try:
            return self._pool.get_nowait()
        except queue.Empty:
            self.torch.cuda.set_device(self.device)
            return {"stream": self.torch.cuda.Stream(device=self.device), "pinned": None}

    def prepare(self, slots: int, nbytes: int) -> None:
        """Make `slots` worker contexts with pinned staging of nbytes each,
        written once and copied once, so that no call pays for pinning pages."""
        ctxs = []
        while len(ctxs) < slots:
            ctxs.append(self._take())
        for ctx in ctxs:
            if nbytes and (ctx["pinned"] is None or ctx["pinned"].numel() < nbytes):
                buf = self.torch.zeros(nbytes, dtype=self.torch.uint8, pin_memory=True)
                ctx["pinned"] = buf
                with self.torch.cuda.stream(ctx["stream"]):
                    self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device).copy_(buf,
                                                                                              non_blocking=True)
                ctx["stream"].synchronize()
        for ctx in ctxs:
            self._pool.put(ctx)

    def _staging(self, ctx: dict, nbytes: int):
        """The context's pinned host buffer of at least nbytes (grown by
        doubling; a call waits for its copy before the context is reused)."""
        buf = ctx["pinned"]
        if buf is None or buf.numel() < nbytes:
            cap = max(nbytes, 2 * (buf.numel() if buf is not None else 1 << 20))
            buf = self.torch.empty(cap, dtype=self.torch.uint8, pin_memory=True)
            ctx["pinned"] = buf
        return buf

    def _to_device(self, ctx: dict, arrays: list, total: int):
        pin = self._staging(ctx, max(total, 1))
        if total:
            np.concatenate(arrays, out=pin.numpy()[:total])
        d = self.torch.empty(max(total, 1), dtype=self.torch.uint8, device=self.device)
        d.copy_(pin[: max(total, 1)], non_blocking=True)
        return d

    def plain(self, req: Request):
        torch = self.torch
        ctx = self._take()
        s = ctx["stream"]
        try:
            with torch.cuda.stream(s):
                seqs = self._to_device(ctx, [req.a, req.b], req.bases)
                sa, joined = lor.lor_build_sa(seqs, req.offsets, stream=s)
                lcp, isa = lor.lor_build_lcp(joined, sa, want_isa=req.keep, stream=s)
                ov = lor.lor_longest_overlap(sa, lcp, req.offsets, stream=s)
                state = None
                if req.keep:
                    rmq = lor.lor_rmq_compact_build(lcp, stream=s)
                    state = {"lcp": lcp, "isa": isa, "rmq": rmq}
                s.synchronize()
        finally:
            self._pool.put(ctx)
        return ov, state

    def batch(self, reqs: list):
        """One batched call over every request; returns [(record, state)]."""
        torch = self.torch
        seqs = [x for r in reqs for x in (r.a, r.b)]
        offs = np.concatenate([[0], np.cumsum([x.size for x in seqs])]).astype(np.int64)
        keep = any(r.keep for r in reqs)
        ctx = self._take()
        s = ctx["stream"]
        try:
            with torch.cuda.stream(s):
                d = self._to_device(ctx, seqs, int(offs[-1]))
                if keep:
                    out, lcp, isa = lor.lor_longest_overlap_batched_state(d, offs, stream=s, plan=self.plan)
                else:
                    out = lor.lor_longest_overlap_batched(d, offs, stream=s, plan=self.plan)
                recs = lor.records_to_tuples(out)   # the call synchronised the stream
                states = [None] * len(reqs)
                if keep:
                    starts = lor.pair_starts(offs)
                    for i, r in enumerate(reqs):
                        if r.keep:
                            s0, s1 = int(starts[i]), int(starts[i + 1])
                            plcp = lcp[s0:s1].clone()
                            pisa = isa[s0:s1] - s0
                            states[i] = {"lcp": plcp, "isa": pisa,
                                         "rmq": lor.lor_rmq_compact_build(plcp, stream=s)}
                    s.synchronize()
        finally:
            self._pool.put(ctx)
        return list(zip(recs, states))

    def followup(self, req: Request, state: dict):
        torch = self.torch
        ctx = self._take()
        s = ctx["stream"]
        try:
            with torch.cuda.stream(s):
                qi = torch.from_numpy(np.ascontiguousarray(req.followup[0], dtype=np.int32)).to(self.device)
                qj = torch.from_numpy(np.ascontiguousarray(req.followup[1], dtype=np.int32)).to(self.device)
                got, _ = lor.lor_rmq_query(state["rmq"], state["lcp"], state["isa"], 1, qi, qj, stream=s)
                res = got.cpu().numpy()
                s.synchronize()
        finally:
            self._pool.put(ctx)
        return res


class Server:
    # Batches of at most 16 pairs and 24M bases on 4 slots: on a backlog of
    # the serving mix this gave the same throughput as larger batches (about
    # 2,100 pairs/s on MI355X) at the lowest median latency.
    def __init__(self, runner=None, budget_bytes: int = 200 << 30, slots: int = 4, batch_max: int = 16,
                 batch_bases: int = 24 << 20, batching: bool = True):
        self.runner = runner if runner is not None else GpuRunner()
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.batch_max = int(batch_max)
        self.batch_bases = int(batch_bases)
        self.batching = batching
        self.in_use = 0
        self.peak_in_use = 0
        self.waits_for_memory = 0
        self.state = {}                              # rid -> resident tensors

    @staticmethod
    def _item_bytes(kind, group):
        if kind == "plain":
            return plain_bytes(group[0].bases, group[0].keep)
        if kind == "batch":
            keep = [r for r in group if r.keep]
            return batch_bytes(sum(r.bases for r in group), len(group), bool(keep)) + sum(
                resident_bytes(r.bases) for r in keep)
        return 0

    # ------------------------------------------------------------ the loop
    def run(self, requests: list, time_scale: float = 1.0) -> dict:
        """Serve `requests` (arrival times in seconds) in real time. Returns stats."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        queue = []            # arrived requests, oldest first
        solo = []             # requests of a failed batch, each to be retried alone
        followups = []        # follow-up batches that are due, oldest first
        timers = []           # (time, seq, request) follow-ups becoming due
        running = {}
        seq = 0
        nxt = 0
        done = 0
        total = len(reqs)
        fol_total = sum(1 for r in reqs if r.keep and r.followup is not None)
        fol_done = 0
        blocked = False       # the oldest queued request is waiting for memory
        prepare = getattr(self.runner, "prepare", None)
        if prepare is not None:
            prepare(self.slots, self.batch_bases if self.batching else max((r.bases for r in reqs), default=0))
        pool = ThreadPoolExecutor(max_workers=self.slots)
        t0 = time.perf_counter()

        def now():
            return (time.perf_counter() - t0) / time_scale

        def reject(r, t):
            nonlocal done, fol_total
            r.rejected = True
            r.t_result = t
            if r.keep and r.followup is not None:
                fol_total -= 1
            done += 1

        def next_work(t):
            """The next item to start, within the free budget, or None."""
            nonlocal blocked
            if followups:
                return "followup", [followups.pop(0)], 0
            while solo:
                kind = "batch" if self.batching else "plain"
                nbytes = self._item_bytes(kind, solo[:1])
                if nbytes > self.budget:
                    reject(solo.pop(0), t)
                    continue
                if self.in_use + nbytes > self.budget:
                    return None
                return kind, [solo.pop(0)], nbytes
            while queue:
                kind = "batch" if self.batching else "plain"
                first = self._item_bytes(kind, queue[:1])
                if first > self.budget:            # can never fit: reject
                    reject(queue.pop(0), t)
                    continue
                if self.in_use + first > self.budget:
                    if not blocked:
                        self.waits_for_memory += 1
                        blocked = True
                    return None
                blocked = False
                k = 1
                nbytes = first
                if self.batching:
                    r0 = queue[0]
                    bases, keep, res = r0.bases, r0.keep, resident_bytes(r0.bases) if r0.keep else 0
                    while k < len(queue) and k < self.batch_max and bases + queue[k].bases <= self.batch_bases:
                        r = queue[k]
                        nb, nk = bases + r.bases, keep or r.keep
                        nres = res + (resident_bytes(r.bases) if r.keep else 0)
                        need = batch_bytes(nb, k + 1, nk) + nres
                        if self.in_use + need > self.budget:
                            break
                        bases, keep, res, nbytes = nb, nk, nres, need
                        k += 1
                group = queue[:k]
                del queue[:k]
                return kind, group, nbytes
            return None

        try:
            while done < total or fol_done < fol_total or running:
                t = now()
                while nxt < total and reqs[nxt].arrival <= t:
                    queue.append(reqs[nxt])
                    nxt += 1
                while timers and timers[0][0] <= t:
                    _, _, r = heapq.heappop(timers)
                    r.t_followup_arrival = t
                    followups.append(r)
                # start work while slots and memory allow
                while len(running) < self.slots:
                    item = next_work(t)
                    if item is None:
                        break
                    kind, group, nbytes = item
                    self.in_use += nbytes
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    if kind == "plain":
                        fut = pool.submit(self.runner.plain, group[0])
                    elif kind == "batch":
                        fut = pool.submit(self.runner.batch, group)
                    else:
                        fut = pool.submit(self.runner.followup, group[0], self.state[group[0].rid])
                    running[fut] = (kind, group, nbytes)
                finished = [f for f in running if f.done()]
                for f in finished:
                    kind, group, nbytes = running.pop(f)
                    err = f.exception()
                    res = None if err is not None else f.result()
                    t_end = now()
                    self.in_use -= nbytes
                    if err is not None:
                        if kind == "followup":
                            r = group[0]
                            r.error = f"follow-up: {err}"
                            r.t_followup = t_end
                            self.state.pop(r.rid, None)
                            self.in_use -= resident_bytes(r.bases)
                            fol_done += 1
                        elif len(group) > 1:
                            solo.extend(group)          # find the request that fails
                        else:
                            r = group[0]
                            r.error = str(err)
                            r.t_result = t_end
                            done += 1
                            if r.keep and r.followup is not None:
                                fol_total -= 1
                        continue
                    if kind == "followup":
                        r = group[0]
                        r.followup_result = res
                        r.t_followup = t_end
                        self.state.pop(r.rid, None)
                        self.in_use -= resident_bytes(r.bases)
                        fol_done += 1
                        continue
                    outs = [res] if kind == "plain" else res
                    for r, (rec, state) in zip(group, outs):
                        r.result = rec
                        r.t_result = t_end
                        r.batched = kind == "batch"
                        done += 1
                        if r.keep and r.followup is not None:
                            self.state[r.rid] = state
                            self.in_use += resident_bytes(r.bases)
                            seq += 1
                            heapq.heappush(timers, (t_end + r.followup_delay, seq, r))
                if not finished:
                    time.sleep(0.0002)
        finally:
            pool.shutdown(wait=True)
        wall = now()
        served = [r for r in reqs if not r.rejected and r.error is None]
        lat = np.array([r.t_result - r.arrival for r in served]) * 1e3
        flat = np.array([r.t_followup - r.t_followup_arrival for r in reqs if r.t_followup is not None]) * 1e3
        nq = sum(r.followup[0].size for r in reqs if r.t_followup is not None)
        # time to the last pair result (the run itself also waits for follow-up batches)
        rspan = max((r.t_result for r in served), default=0.0) - (reqs[0].arrival if reqs else 0.0)
        return {
            "requests": total, "rejected": sum(r.rejected for r in reqs),
            "failed": sum(r.error is not None and not r.rejected and r.result is None for r in reqs),
            "wall_s": round(wall, 3),
            "pairs_per_s": round(len(served) / wall, 1) if wall > 0 else None,
            "results_s": round(rspan, 4),
            "result_pairs_per_s": round(len(served) / rspan, 1) if rspan > 0 else None,
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
            "batched_requests": sum(r.batched for r in reqs),
            "followups": int(flat.size),
            "followup_p50_ms": round(float(np.percentile(flat, 50)), 3) if flat.size else None,
            "followup_p99_ms": round(float(np.percentile(flat, 99)), 3) if flat.size else None,
            "followup_queries_per_s": round(nq / wall, 1) if wall > 0 else None,
            "peak_admitted_bytes": int(self.peak_in_use),
            "waits_for_memory": int(self.waits_for_memory),
            "budget_bytes": self.budget, "slots": self.slots,
        }


def make_requests(seed: int = 5, count: int = 400, qps: float = 100.0, lo: float = 1e4, hi: float = 4e6,
                  keep_frac: float = 0.3, queries: int = 10_000, followup_mean: float = 0.05) -> list:
    """Poisson arrivals at `qps`; each sequence length log-uniform in [lo, hi]
    with the noncoding-like generator; `keep_frac` of the requests keep state
    and send `queries` uniform suffix-pair queries after an exponential delay
    of mean `followup_mean` seconds."""
    from . import synth
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / qps))
        la = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        lb = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        a = synth.noncoding_like(rng, la)
        b = synth.noncoding_like(rng, lb)
        keep = bool(rng.random() < keep_frac)
        fol = None
        delay = 0.0
        if keep:
            n = la + lb + 2
            fol = (rng.integers(0, n, size=queries).astype(np.int32), rng.integers(0, n, size=queries).astype(np.int32))
            delay = float(rng.exponential(followup_mean))
        out.append(Request(i, a, b, t, keep, fol, delay))
    return out


def main():
    """The serving scenario on cuda:0: capacity on a backlog, then Poisson
    arrivals at a fraction of it; prints one JSON line of stats. Every request
    is generated before the first GPU call, and the phases (warm-up, capacity,
    Poisson run) are half a second apart, so a kernel trace of the run splits
    into them at its idle gaps."""
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="continuous-batching serving run on one GPU")
    ap.add_argument("--backlog", type=int, default=96, help="requests of the capacity run (all at t = 0)")
    ap.add_argument("--count", type=int, default=400, help="requests of the Poisson run")
    ap.add_argument("--load", type=float, default=0.7, help="offered rate as a fraction of the capacity")
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args()
    from . import autotune
    warm = make_requests(seed=args.seed + 200, count=16, qps=1e9)
    backlog = make_requests(seed=args.seed + 100, count=args.backlog, qps=1e9)
    for r in warm + backlog:
        r.arrival = 0.0
    reqs = make_requests(seed=args.seed, count=args.count, qps=1.0)   # arrival times rescaled below
    lor.lib()
    autotune.load_tuned_plan()
    runner = GpuRunner(plan=autotune.load_batched_plan())
    Server(runner=runner, batch_max=4).run(warm)
    time.sleep(0.5)
    cap = Server(runner=runner).run(backlog)
    qps = args.load * cap["result_pairs_per_s"]
    print(f"capacity: {cap['result_pairs_per_s']} pairs/s; offering {qps:.1f} requests/s", file=sys.stderr,
          flush=True)
    for r in reqs:   # exponential gaps scale with 1 / qps
        r.arrival /= qps
    time.sleep(0.5)
    stats = Server(runner=runner).run(reqs)
    stats["capacity_pairs_per_s"] = cap["result_pairs_per_s"]
    stats["capacity_p50_ms"] = cap["p50_ms"]
    stats["offered_qps"] = round(qps, 1)
    print(json.dumps(stats))


if __name__ == "__main__":
    main()
