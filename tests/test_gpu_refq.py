"""One reference against many query sequences (the shape of Section V's
experiments): every record against the O(nm) DP oracle (length and query
offset exactly; the reference offset must hold the same substring)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1404_3448_amd import lor, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def run(ref, queries):
    seqs = [ref] + list(queries)
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    cat = np.concatenate(seqs) if offs[-1] else np.zeros(1, np.uint8)
    d = torch.from_numpy(np.ascontiguousarray(cat)).cuda()
    return lor.records_to_tuples(lor.lor_longest_overlap_ref(d, offs))


def check(ref, queries, got):
    assert len(got) == len(queries)
    for q, (query, rec) in enumerate(zip(queries, got)):
        L, xa, yb = oracle.lcs_dp(query, ref)      # first maximum: smallest query offset
        length, seq_p, off_p, seq_q, off_q = rec
        assert length == L, (q, rec, (L, xa, yb))
        if L == 0:
            assert rec == (0, -1, -1, -1, -1), q
            continue
        assert (seq_p, seq_q, off_p) == (q + 1, 0, xa), (q, rec, (L, xa, yb))
        assert 0 <= off_q <= ref.size - L
        assert np.array_equal(ref[off_q:off_q + L], query[xa:xa + L]), q


def test_ref_closed_forms():
    ref = synth.encode("ATTGCTACGGA")
    queries = [synth.encode("GCTA"), synth.encode("CCCC"), np.zeros(0, np.uint8), ref.copy(),
               synth.encode("TTGCTACGGAT"), synth.encode("A")]
    got = run(ref, queries)
    check(ref, queries, got)
    assert got[0][0] == 4 and got[3][0] == ref.size and got[2][0] == 0


@pytest.mark.parametrize("seed", range(8))
def test_ref_random_small(seed):
    rng = np.random.default_rng(900 + seed)
    alpha = int(rng.integers(1, 5))
    ref = rng.integers(0, alpha, size=int(rng.integers(0, 400)), dtype=np.uint8)
    queries = []
    for _ in range(int(rng.integers(1, 120))):
        q = rng.integers(0, alpha, size=int(rng.integers(0, 120)), dtype=np.uint8)
        if ref.size > 20 and q.size > 10 and rng.random() < 0.5:
            s = int(rng.integers(0, ref.size - 10))
            q = np.concatenate([q[: q.size // 2], ref[s:s + int(rng.integers(3, 60))], q[q.size // 2:]])
        queries.append(q)
    say("refq", seed, ref.size, len(queries))
    check(ref, queries, run(ref, queries))


def test_ref_many_tiny_queries():
    """20,000 queries of 0-3 bases: a 64-position bucket of the sequence
    lookup then holds dozens of query starts, so every lookup searches
    inside its bucket, and empty queries are pure separators."""
    rng = np.random.default_rng(911)
    ref = rng.integers(0, 4, size=300, dtype=np.uint8)
    queries = [rng.integers(0, 4, size=int(rng.integers(0, 4)), dtype=np.uint8) for _ in range(20000)]
    check(ref, queries, run(ref, queries))


def test_ref_noncoding_many_queries():
    rng = synth.rng_for(77)
    ref = synth.noncoding_like(rng, 100_000)
    queries = []
    for i in range(400):
        q = synth.noncoding_like(rng, int(rng.integers(0, 3000)))
        if q.size > 100 and i % 3:
            s = int(rng.integers(0, ref.size - 2000))
            seg = synth.mutate(rng, ref[s:s + int(rng.integers(20, 1500))].copy(), 0.01)
            p = int(rng.integers(0, q.size))
            q = np.concatenate([q[:p], seg, q[p:]])
        queries.append(q)
    got = run(ref, queries)
    check(ref, queries[:12], got[:12])          # the DP oracle on a sample of the queries
    # every query against the oracle's scan of its (query, reference) pair, in CPU
    # worker processes: the length and the smallest query offset are unique, the
    # reference offset must hold the same substring
    import oracle_pool
    want = oracle_pool.pairs_overlap([(q, ref) for q in queries])
    for q, (query, (L, _, op, _, _)) in enumerate(zip(queries, want)):
        assert got[q][0] == L, q
        if L:
            assert got[q][2] == op, q
            assert np.array_equal(query[op:op + L], ref[got[q][4]:got[q][4] + L]), q


def test_ref_rejects_bad_base():
    ref = synth.encode("ACGTACGT")
    bad = np.array([0, 1, 7, 2], np.uint8)
    with pytest.raises(lor.LorError) as e:
        run(ref, [synth.encode("ACG"), bad])
    assert e.value.status == lor.LOR_EALPHABET
