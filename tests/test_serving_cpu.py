"""Host logic of the serving loop with a fake runner (no GPU): continuous
batching, admission by the HBM budget (and waiting for memory), rejection of
requests that can never fit, follow-ups on resident state."""
import threading
import time

import numpy as np

from paper_1404_3448_amd import serve


class FakeRunner:
    """Sleeps in proportion to the work and returns a tag instead of a result."""

    def __init__(self):
        self.lock = threading.Lock()
        self.calls = []

    def plain(self, req):
        with self.lock:
            self.calls.append(("plain", req.rid))
        time.sleep(1e-9 * req.bases + 0.001)
        return ("plain", req.rid), ({"rid": req.rid} if req.keep else None)

    def batch(self, reqs):
        with self.lock:
            self.calls.append(("batch", tuple(r.rid for r in reqs)))
        time.sleep(1e-9 * sum(r.bases for r in reqs) + 0.002)
        return [(("batch", r.rid), ({"rid": r.rid} if r.keep else None)) for r in reqs]

    def followup(self, req, state):
        assert state == {"rid": req.rid}
        with self.lock:
            self.calls.append(("followup", req.rid))
        return np.full(req.followup[0].size, req.rid, dtype=np.int32)


def mk(rid, na, nb, t, keep=False):
    rng = np.random.default_rng(rid)
    a = rng.integers(0, 4, size=na, dtype=np.uint8)
    b = rng.integers(0, 4, size=nb, dtype=np.uint8)
    fol = (np.zeros(7, np.int32), np.zeros(7, np.int32)) if keep else None
    return serve.Request(rid, a, b, t, keep, fol, 0.003 if keep else 0.0)


def test_every_request_is_served_in_batches():
    # bursts of 10 arrivals: more requests wait than there are free slots
    reqs = [mk(i, 500 if i % 3 else 600_000, 400, 0.004 * (i // 10), keep=(i % 5 == 0)) for i in range(40)]
    runner = FakeRunner()
    srv = serve.Server(runner=runner, slots=3, batch_max=8, batch_bases=2_000_000)
    stats = srv.run(reqs)
    assert stats["requests"] == 40 and stats["rejected"] == 0
    for r in reqs:
        assert r.result == ("batch", r.rid)
        assert r.t_result >= r.arrival
        if r.keep:
            assert np.all(r.followup_result == r.rid)
            assert r.t_followup_arrival >= r.t_result
    batches = [c[1] for c in runner.calls if c[0] == "batch"]
    assert sorted(x for b in batches for x in b) == list(range(40))
    assert max(len(b) for b in batches) > 1 and all(len(b) <= 8 for b in batches)
    assert all(sum(reqs[x].bases for x in b) <= 2_000_000 or len(b) == 1 for b in batches)
    for b in batches:                              # oldest first, in arrival order
        assert list(b) == sorted(b)
    assert stats["batched_requests"] == 40
    assert stats["followups"] == sum(r.keep for r in reqs)
    assert srv.in_use == 0 and not srv.state


def test_batches_wait_for_memory():
    reqs = [mk(i, 40_000, 40_000, 0.0, keep=(i % 2 == 0)) for i in range(12)]
    one = serve.Server._item_bytes("batch", reqs[:1])
    runner = FakeRunner()
    srv = serve.Server(runner=runner, budget_bytes=int(2.2 * one), slots=4, batch_max=3)
    stats = srv.run(reqs)
    assert stats["rejected"] == 0 and stats["waits_for_memory"] > 0
    assert srv.peak_in_use <= srv.budget
    assert all(r.result == ("batch", r.rid) for r in reqs)
    assert srv.in_use == 0 and not srv.state


def test_budget_limits_concurrency_and_rejects_oversized():
    small = serve.plain_bytes(100_000, False)
    big = mk(99, 3_000_000, 3_000_000, 0.0)
    reqs = [mk(i, 50_000, 50_000, 0.0) for i in range(6)] + [big]
    runner = FakeRunner()
    srv = serve.Server(runner=runner, budget_bytes=int(2.5 * small), slots=4, batching=False)
    stats = srv.run(reqs)
    assert stats["rejected"] == 1 and big.rejected and big.result is None
    assert srv.peak_in_use <= srv.budget
    assert srv.peak_in_use >= 2 * small          # two fit at once, never three
    assert all(r.result == ("plain", r.rid) for r in reqs[:6])


def test_byte_accounting_matches_size_queries():
    from paper_1404_3448_amd import lor
    n = 1000 + 2
    ws = max(lor.lor_build_sa_workspace(1000, 2), lor.lor_build_lcp_workspace(n), lor.lor_longest_overlap_workspace(n, 2))
    assert serve.plain_bytes(1000, False) == 1000 + n + 8 * n + ws
    assert serve.plain_bytes(1000, True) - serve.plain_bytes(1000, False) == 4 * n + lor.lor_rmq_compact_bytes(n)
    assert serve.resident_bytes(1000) == 8 * n + lor.lor_rmq_compact_bytes(n)


class FailingRunner(FakeRunner):
    """Fails every call whose requests include `bad`."""

    def __init__(self, bad):
        super().__init__()
        self.bad = bad

    def batch(self, reqs):
        if any(r.rid == self.bad for r in reqs):
            with self.lock:
                self.calls.append(("fail", tuple(r.rid for r in reqs)))
            raise RuntimeError("lor_longest_overlap_batched: status 2 (base outside A,C,G,T (0..3))")
        return super().batch(reqs)


def test_a_failing_request_fails_alone():
    reqs = [mk(i, 3000, 2000, 0.0, keep=(i % 4 == 0)) for i in range(24)]
    runner = FailingRunner(bad=9)
    srv = serve.Server(runner=runner, slots=2, batch_max=8)
    stats = srv.run(reqs)
    assert stats["failed"] == 1 and stats["rejected"] == 0
    assert reqs[9].result is None and "status 2" in reqs[9].error
    for r in reqs:
        if r.rid != 9:
            assert r.result == ("batch", r.rid) and r.error is None
            if r.keep:
                assert np.all(r.followup_result == r.rid)
    fails = [c[1] for c in runner.calls if c[0] == "fail"]
    assert len(fails) == 2 and fails[-1] == (9,)     # the batch, then request 9 alone
    assert srv.in_use == 0 and not srv.state
