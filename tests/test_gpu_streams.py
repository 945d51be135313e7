"""Calls on a stream other than torch's current one: the binding allocates
workspaces and outputs on that stream, so an allocation made on the current
stream right after the call cannot be handed a workspace the call's kernels
still use. Results are checked against the oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_1404_3448_amd import lor, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def test_side_stream_calls_then_allocate_on_current_stream():
    w = synth.tiny_pair(seed=12, n=400_000, planted_len=700)
    say("side stream:", w.joined_length, "ranks")
    d = torch.from_numpy(w.concat).cuda()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    sa, joined = lor.lor_build_sa(d, w.offsets, stream=side)
    lcp, isa = lor.lor_build_lcp(joined, sa, want_isa=True, stream=side)   # returns while its kernels run
    # allocations on the current stream, right away, written at once
    junk = [torch.full((w.joined_length * 8,), -7, dtype=torch.int32, device="cuda") for _ in range(4)]
    rmq = lor.lor_rmq_build(lcp, stream=side)
    n = w.joined_length
    rng = np.random.default_rng(3)
    qi = rng.integers(0, n, size=5000).astype(np.int32)
    qj = rng.integers(0, n, size=5000).astype(np.int32)
    with torch.cuda.stream(side):
        tqi, tqj = torch.from_numpy(qi).cuda(), torch.from_numpy(qj).cuda()
    got, _ = lor.lor_rmq_query(rmq, lcp, isa, 1, tqi, tqj, stream=side)
    junk += [torch.full((w.joined_length * 8,), -9, dtype=torch.int32, device="cuda") for _ in range(4)]
    ov = lor.lor_longest_overlap(sa, lcp, w.offsets, stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    assert all(int(j[0]) in (-7, -9) for j in junk)
    joined_o = oracle.join(w.concat, w.offsets)
    sa_o = oracle.suffix_array(joined_o)
    lcp_o = oracle.lcp(joined_o, sa_o)
    assert np.array_equal(sa.cpu().numpy(), sa_o)
    assert np.array_equal(lcp.cpu().numpy(), lcp_o)
    isa_o = np.empty_like(sa_o)
    isa_o[sa_o] = np.arange(n, dtype=sa_o.dtype)
    assert np.array_equal(isa.cpu().numpy(), isa_o)
    assert np.array_equal(got.cpu().numpy(), oracle.pair_queries(joined_o, qi, qj))
    assert ov == oracle.overlap(sa_o, lcp_o, w.offsets)


def test_side_stream_sort_pairs_and_batched():
    rng = np.random.default_rng(21)
    n = 3_000_000
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.int32)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        k = torch.from_numpy(keys.view(np.int32)).cuda()
        v = torch.from_numpy(vals).cuda()
    lor.lor_sort_pairs_u32(k, v, 0, 32, stream=side)          # its workspace is freed on return
    junk = torch.full((n * 4,), 5, dtype=torch.int32, device="cuda")
    pairs = [(synth.random_text(40 + i, 3000 + 17 * i), synth.random_text(90 + i, 2500 + 11 * i)) for i in range(20)]
    seqs = [s for ab in pairs for s in ab]
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    with torch.cuda.stream(side):
        d = torch.from_numpy(np.concatenate(seqs)).cuda()
    out = lor.lor_longest_overlap_batched(d, offs, stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    assert int(junk[-1]) == 5
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(k.cpu().numpy().view(np.uint32), keys[order])
    assert np.array_equal(v.cpu().numpy(), vals[order])
    recs = lor.records_to_tuples(out)
    for p, (a, b) in enumerate(pairs):
        o = np.array([0, a.size, a.size + b.size], np.int64)
        j = oracle.join(np.concatenate([a, b]), o)
        s_ = oracle.suffix_array(j)
        assert recs[p] == oracle.overlap(s_, oracle.lcp(j, s_), o), p
