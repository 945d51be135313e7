"""Serving loop for longest-overlap requests on one GPU (continuous batching).

Requests (a pair of DNA sequences, an arrival time, and optionally a batch of
follow-up suffix-pair lcp queries) arrive over time. The loop

* admits work while an HBM budget holds, charging every request the exact
  bytes the library's size queries give (workspace, outputs, and, for
  requests that keep state, the resident LCP/ISA/sparse table);
* runs admitted work concurrently, each worker thread on its own HIP stream,
  so requests that arrive while others are on the GPU start as soon as a slot
  and memory free up and their kernels overlap on the device;
* coalesces small requests into mini-batches for the batched entry point and
  runs large requests (and every request that keeps state) on the plain path;
* keeps SA-derived state resident for the requests that ask for it (LCP,
  ISA and the compact block sparse table, about 8.4 bytes per base), answers
  their follow-up query batch when it arrives, then frees it;
* records arrival-to-result latency per request and per follow-up batch.

All GPU work goes through the C-ABI (paper_1404_3448_amd.lor); nothing here
computes on the CPU besides bookkeeping.
"""
from __future__ import annotations

import ctypes
import heapq
import threading
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


def batch_bytes(total_bases: int, pairs: int) -> int:
    return int(total_bases + lor.lor_longest_overlap_batched_workspace(total_bases, pairs)
               + pairs * ctypes.sizeof(lor.lor_overlap))


class GpuRunner:
    """Device work of the serving loop; every call runs on the calling
    thread's own HIP stream (default priority)."""

    def __init__(self, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self._tls = threading.local()
        lor.lib()

    def _stream(self):
        s = getattr(self._tls, "stream", None)
        if s is None:
            self.torch.cuda.set_device(self.device)
            s = self.torch.cuda.Stream(device=self.device)
            self._tls.stream = s
        return s

    def plain(self, req: Request):
        torch = self.torch
        s = self._stream()
        with torch.cuda.stream(s):
            seqs = torch.from_numpy(np.concatenate([req.a, req.b]) if req.bases else np.zeros(1, np.uint8))
            seqs = seqs.to(self.device, non_blocking=False)
            sa, joined = lor.lor_build_sa(seqs, req.offsets, stream=s)
            lcp, isa = lor.lor_build_lcp(joined, sa, want_isa=req.keep, stream=s)
            ov = lor.lor_longest_overlap(sa, lcp, req.offsets, stream=s)
            state = None
            if req.keep:
                rmq = lor.lor_rmq_compact_build(lcp, stream=s)
                state = {"lcp": lcp, "isa": isa, "rmq": rmq}
            s.synchronize()
        return ov, state

    def batch(self, reqs: list):
        torch = self.torch
        s = self._stream()
        with torch.cuda.stream(s):
            seqs = [x for r in reqs for x in (r.a, r.b)]
            offs = np.concatenate([[0], np.cumsum([x.size for x in seqs])]).astype(np.int64)
            cat = np.concatenate(seqs) if offs[-1] else np.zeros(1, np.uint8)
            d = torch.from_numpy(cat).to(self.device, non_blocking=False)
            out = lor.lor_longest_overlap_batched(d, offs, stream=s)
            recs = lor.records_to_tuples(out)   # synchronises the copy
        return recs

    def followup(self, req: Request, state: dict):
        torch = self.torch
        s = self._stream()
        with torch.cuda.stream(s):
            qi = torch.from_numpy(np.ascontiguousarray(req.followup[0], dtype=np.int32)).to(self.device)
            qj = torch.from_numpy(np.ascontiguousarray(req.followup[1], dtype=np.int32)).to(self.device)
            got, _ = lor.lor_rmq_query(state["rmq"], state["lcp"], state["isa"], 1, qi, qj, stream=s)
            res = got.cpu().numpy()
            s.synchronize()
        return res


class Server:
    def __init__(self, runner=None, budget_bytes: int = 200 << 30, slots: int = 4, small_bases: int = 400_000,
                 batch_max: int = 64, batch_wait: float = 0.002, batching: bool = True):
        self.runner = runner if runner is not None else GpuRunner()
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.small = int(small_bases)
        self.batch_max = int(batch_max)
        self.batch_wait = float(batch_wait)
        self.batching = batching
        self.in_use = 0
        self.peak_in_use = 0
        self.state = {}                              # rid -> resident tensors

    # ------------------------------------------------------------ the loop
    def run(self, requests: list, time_scale: float = 1.0) -> dict:
        """Serve `requests` (arrival times in seconds) in real time. Returns stats."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        pending = []          # arrived, waiting for admission (FIFO)
        smalls = []           # arrived small requests waiting to form a batch
        timers = []           # (time, seq, kind, payload) follow-ups becoming due
        running = {}
        seq = 0
        nxt = 0
        done = 0
        total = len(reqs)
        fol_total = sum(1 for r in reqs if r.keep and r.followup is not None)
        fol_done = 0
        pool = ThreadPoolExecutor(max_workers=self.slots)
        t0 = time.perf_counter()

        def now():
            return (time.perf_counter() - t0) / time_scale

        def admit(item_bytes):
            if self.in_use + item_bytes <= self.budget:
                self.in_use += item_bytes
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                return True
            return False

        try:
            while done < total or fol_done < fol_total or running:
                t = now()
                while nxt < total and reqs[nxt].arrival <= t:
                    r = reqs[nxt]
                    nxt += 1
                    if self.batching and not r.keep and r.bases <= self.small:
                        smalls.append(r)
                    else:
                        pending.append(("plain", [r], plain_bytes(r.bases, r.keep)))
                if smalls and (len(smalls) >= self.batch_max or t - smalls[0].arrival >= self.batch_wait
                               or nxt >= total):
                    group = smalls[: self.batch_max]
                    del smalls[: len(group)]
                    pending.append(("batch", group, batch_bytes(sum(r.bases for r in group), len(group))))
                while timers and timers[0][0] <= t:
                    _, _, r = heapq.heappop(timers)
                    r.t_followup_arrival = t
                    pending.append(("followup", [r], 0))
                # admit in arrival order while slots and memory allow
                while pending and len(running) < self.slots:
                    kind, group, nbytes = pending[0]
                    if nbytes > self.budget:           # can never fit: reject
                        pending.pop(0)
                        for r in group:
                            r.rejected = True
                            r.t_result = t
                            if r.keep and r.followup is not None:
                                fol_total -= 1
                        done += len(group)
                        continue
                    if not admit(nbytes):
                        break
                    pending.pop(0)
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
                    res = f.result()
                    t_end = now()
                    self.in_use -= nbytes
                    if kind == "plain":
                        r = group[0]
                        r.result, state = res
                        r.t_result = t_end
                        done += 1
                        if r.keep and r.followup is not None:
                            self.state[r.rid] = state
                            self.in_use += resident_bytes(r.bases)
                            seq += 1
                            heapq.heappush(timers, (t_end + r.followup_delay, seq, r))
                    elif kind == "batch":
                        for r, rec in zip(group, res):
                            r.result = rec
                            r.t_result = t_end
                            r.batched = True
                        done += len(group)
                    else:
                        r = group[0]
                        r.followup_result = res
                        r.t_followup = t_end
                        self.state.pop(r.rid, None)
                        self.in_use -= resident_bytes(r.bases)
                        fol_done += 1
                if not finished:
                    time.sleep(0.0002)
        finally:
            pool.shutdown(wait=True)
        wall = now()
        served = [r for r in reqs if not r.rejected]
        lat = np.array([r.t_result - r.arrival for r in served]) * 1e3
        flat = np.array([r.t_followup - r.t_followup_arrival for r in reqs if r.t_followup is not None]) * 1e3
        nq = sum(r.followup[0].size for r in reqs if r.t_followup is not None)
        return {
            "requests": total, "rejected": total - len(served), "wall_s": round(wall, 3),
            "pairs_per_s": round(len(served) / wall, 1) if wall > 0 else None,
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
            "batched_requests": sum(r.batched for r in reqs),
            "followups": int(flat.size),
            "followup_p50_ms": round(float(np.percentile(flat, 50)), 3) if flat.size else None,
            "followup_p99_ms": round(float(np.percentile(flat, 99)), 3) if flat.size else None,
            "followup_queries_per_s": round(nq / wall, 1) if wall > 0 else None,
            "peak_admitted_bytes": int(self.peak_in_use),
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
