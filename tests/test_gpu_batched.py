"""Batched longest overlap (many pairs, one DC3 run) against the oracle, pair by pair."""
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1404_3448_amd import lor, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def flat(pairs):
    seqs = [s for ab in pairs for s in ab]
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    cat = np.concatenate(seqs) if offs[-1] else np.zeros(1, np.uint8)
    return torch.from_numpy(np.ascontiguousarray(cat)).cuda(), offs


def oracle_pair(a, b):
    offs = np.array([0, a.size, a.size + b.size], np.int64)
    joined = oracle.join(np.concatenate([a, b]) if a.size + b.size else np.zeros(0, np.uint8), offs)
    sa = oracle.suffix_array(joined)
    return oracle.overlap(sa, oracle.lcp(joined, sa), offs)


def run_batched(pairs):
    d, offs = flat(pairs)
    out = lor.lor_longest_overlap_batched(d, offs)
    return lor.records_to_tuples(out)


def test_batched_closed_forms(golden):
    cases = golden["overlap_closed_forms"]["cases"]
    pairs = [(synth.encode(c["a"]), synth.encode(c["b"])) for c in cases]
    assert [list(r) for r in run_batched(pairs)] == [c["expect"] for c in cases]


@pytest.mark.parametrize("seed", range(6))
def test_batched_random_pairs(seed):
    rng = np.random.default_rng(500 + seed)
    P = int(rng.integers(1, 400))
    pairs = []
    for _ in range(P):
        alpha = int(rng.integers(1, 5))
        a = rng.integers(0, alpha, size=int(rng.integers(0, 600)), dtype=np.uint8)
        b = rng.integers(0, alpha, size=int(rng.integers(0, 600)), dtype=np.uint8)
        if a.size > 20 and b.size > 20 and rng.random() < 0.5:
            s = int(rng.integers(0, a.size - 10))
            seg = a[s:s + int(rng.integers(5, 200))]
            b = np.concatenate([b[: b.size // 3], seg, b[b.size // 3:]])
        pairs.append((a, b))
    say("batched", seed, P)
    got = run_batched(pairs)
    for p, (a, b) in enumerate(pairs):
        assert got[p] == oracle_pair(a, b), p


def test_batched_tiny_pairs_brute_force():
    rng = np.random.default_rng(77)
    pairs = [(rng.integers(0, 3, size=int(rng.integers(0, 12)), dtype=np.uint8),
              rng.integers(0, 3, size=int(rng.integers(0, 12)), dtype=np.uint8)) for _ in range(4096)]
    got = run_batched(pairs)
    for p, (a, b) in enumerate(pairs):
        assert got[p] == brute.longest_overlap([a, b]), p


def test_batched_many_minimal_pairs():
    """8000 pairs of 0-2 bases: a 4096-rank tile then spans more pairs than a
    workgroup keeps in LDS, so the join, the per-pair maximum, the run pass and
    the level-0 naming all take their search-over-all-pairs paths."""
    rng = np.random.default_rng(78)
    pairs = [(rng.integers(0, 2, size=int(rng.integers(0, 3)), dtype=np.uint8),
              rng.integers(0, 2, size=int(rng.integers(0, 3)), dtype=np.uint8)) for _ in range(8000)]
    got = run_batched(pairs)
    for p, (a, b) in enumerate(pairs):
        assert got[p] == brute.longest_overlap([a, b]), p


def test_batched_equals_plain_path():
    ws = synth.batched_pairs(seed=11, num_pairs=24, lo=1e3, hi=2e5)
    pairs = [tuple(w.seqs) for w in ws]
    got = run_batched(pairs)
    for p, w in enumerate(ws):
        d = torch.from_numpy(w.concat).cuda()
        plain = lor.longest_overlap_region(d, w.offsets)["overlap"]
        assert got[p] == plain, p
        assert got[p] == oracle_pair(*w.seqs), p


def test_batched_rejects_bad_base():
    d, offs = flat([(np.array([0, 1], np.uint8), np.array([9], np.uint8))])
    with pytest.raises(lor.LorError) as e:
        lor.lor_longest_overlap_batched(d, offs)
    assert e.value.status == lor.LOR_EALPHABET


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_batched_full_size():
    """4096 pairs with log-uniform totals in [1e3, 1e6] (the batched workload
    at full size, 582M bases): every record equals the oracle's for its pair
    (16 CPU worker processes), is well-formed and its two substrings are equal."""
    import oracle_pool
    ws = synth.batched_pairs()
    pairs = [tuple(w.seqs) for w in ws]
    say("batched workload", sum(a.size + b.size for a, b in pairs))
    got = run_batched(pairs)
    say("oracle over every pair")
    want = oracle_pool.pairs_overlap(pairs)
    for p in range(len(pairs)):
        assert got[p] == want[p], p
    for (L, sp, op, sq, oq), (a, b) in zip(got, pairs):
        if L:
            assert (sp, sq) == (0, 1)
            assert np.array_equal(a[op:op + L], b[oq:oq + L])


@pytest.mark.parametrize("seed", range(2))
def test_batched_state_lcp_isa_per_pair(seed):
    """lor_longest_overlap_batched_state: same records as the batched call, and
    each pair's slice of the batch's LCP / ISA equals the oracle's LCP / ISA
    of the pair's own joined text."""
    rng = np.random.default_rng(900 + seed)
    pairs = []
    for _ in range(int(rng.integers(20, 60))):
        la, lb = (int(x) for x in rng.integers(0, 3000, size=2))
        a = synth.noncoding_like(rng, la) if la else np.zeros(0, np.uint8)
        b = synth.noncoding_like(rng, lb) if lb else np.zeros(0, np.uint8)
        if a.size > 100 and b.size > 100:
            s = int(rng.integers(0, a.size - 60))
            b = np.concatenate([b[:50], a[s:s + 60], b[50:]])
        pairs.append((a, b))
    d, offs = flat(pairs)
    say("batched state", seed, len(pairs), int(offs[-1]))
    out, lcp, isa = lor.lor_longest_overlap_batched_state(d, offs)
    recs = lor.records_to_tuples(out)
    assert recs == run_batched(pairs)
    starts = lor.pair_starts(offs)
    assert starts[-1] == lcp.numel()
    lcp, isa = lcp.cpu().numpy(), isa.cpu().numpy()
    for p, (a, b) in enumerate(pairs):
        s0, s1 = int(starts[p]), int(starts[p + 1])
        po = np.array([0, a.size, a.size + b.size], np.int64)
        joined = oracle.join(np.concatenate([a, b]), po)
        sa = oracle.suffix_array(joined)
        assert np.array_equal(lcp[s0:s1], oracle.lcp(joined, sa)), p
        assert np.array_equal(isa[s0:s1] - s0, oracle.isa(sa)), p
        assert recs[p] == oracle.overlap(sa, oracle.lcp(joined, sa), po), p
