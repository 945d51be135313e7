"""Serving on the GPU: every result (and follow-up answer) is the same served
alone and in a concurrent mix of batches, also when the HBM budget makes
batches wait for memory, and equals the oracle."""
import numpy as np
import pytest

import oracle
from paper_1404_3448_amd import lor, serve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def alone(req):
    d = torch.from_numpy(np.concatenate([req.a, req.b])).cuda()
    r = lor.longest_overlap_region(d, req.offsets, want_isa=True)
    fol = None
    if req.keep:
        rmq = lor.lor_rmq_build(r["lcp"])
        got, _ = lor.lor_rmq_query(rmq, r["lcp"], r["isa"], 1, torch.from_numpy(req.followup[0]).cuda(),
                                   torch.from_numpy(req.followup[1]).cuda())
        fol = got.cpu().numpy()
    return r["overlap"], fol


def test_alone_equals_mix():
    reqs = serve.make_requests(seed=5, count=80, qps=400.0, lo=1e3, hi=3e5, queries=2000, followup_mean=0.01)
    srv = serve.Server(slots=4, batch_max=16)
    stats = srv.run(reqs)
    assert stats["rejected"] == 0
    assert stats["batched_requests"] > 0 and stats["followups"] > 0
    for r in reqs:
        ov, fol = alone(r)
        assert r.result == ov, r.rid
        if r.keep:
            assert np.array_equal(r.followup_result, fol), r.rid
    for r in reqs[:6]:
        joined = oracle.join(np.concatenate([r.a, r.b]), r.offsets)
        sa = oracle.suffix_array(joined)
        assert r.result == oracle.overlap(sa, oracle.lcp(joined, sa), r.offsets)
        if r.keep:
            assert np.array_equal(r.followup_result, oracle.pair_queries(joined, *r.followup))


def test_alone_equals_mix_under_memory_pressure():
    reqs = serve.make_requests(seed=8, count=40, qps=2000.0, lo=2e4, hi=2e5, queries=1000, followup_mean=0.005)
    biggest = max(serve.Server._item_bytes("batch", [r]) for r in reqs)
    srv = serve.Server(slots=4, batch_max=4, budget_bytes=int(2.5 * biggest))
    stats = srv.run(reqs)
    assert stats["rejected"] == 0 and stats["waits_for_memory"] > 0
    assert srv.peak_in_use <= srv.budget and srv.in_use == 0
    for r in reqs:
        ov, fol = alone(r)
        assert r.result == ov, r.rid
        if r.keep:
            assert np.array_equal(r.followup_result, fol), r.rid


def test_bad_request_fails_alone_on_the_gpu():
    reqs = serve.make_requests(seed=9, count=12, qps=1e9, lo=2e4, hi=1e5, queries=500, followup_mean=0.002)
    bad = reqs[5]
    bad.a = bad.a.copy()
    bad.a[bad.a.size // 2] = 7                  # not a base
    srv = serve.Server(slots=2, batch_max=6)
    stats = srv.run(reqs)
    assert stats["failed"] == 1 and bad.result is None and "status 2" in bad.error
    for r in reqs:
        if r is not bad:
            ov, fol = alone(r)
            assert r.result == ov, r.rid
            if r.keep:
                assert np.array_equal(r.followup_result, fol), r.rid
