"""All-pairs longest overlap over one joined text: every off-diagonal record
against the O(nm) DP oracle (length and first offset exactly; the second
offset must hold the same substring), symmetry of the lengths, and the
matrix maximum against the single longest overlap."""
import sys

import numpy as np
import pytest

import oracle
from paper_1404_3448_amd import lor, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def matrix(seqs):
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    cat = np.concatenate(seqs) if offs[-1] else np.zeros(1, np.uint8)
    d = torch.from_numpy(np.ascontiguousarray(cat)).cuda()
    r = lor.longest_overlap_region(d, offs)
    recs = lor.records_to_tuples(lor.lor_overlap_matrix(r["sa"], r["lcp"], offs))
    k = len(seqs)
    return [recs[a * k:(a + 1) * k] for a in range(k)], r["overlap"]


def check(seqs):
    M, single = matrix(seqs)
    k = len(seqs)
    for a in range(k):
        assert M[a][a] == (0, -1, -1, -1, -1)
        for b in range(k):
            if a == b:
                continue
            L, xa, xb = oracle.lcs_dp(seqs[a], seqs[b])
            rec = M[a][b]
            assert rec[0] == L, (a, b, rec, (L, xa, xb))
            if L == 0:
                assert rec == (0, -1, -1, -1, -1)
                continue
            assert (rec[1], rec[2], rec[3]) == (a, xa, b), (a, b, rec, (L, xa, xb))
            assert np.array_equal(seqs[b][rec[4]:rec[4] + L], seqs[a][xa:xa + L]), (a, b)
            assert M[b][a][0] == L
    assert max(M[a][b][0] for a in range(k) for b in range(k)) == single[0]


def test_matrix_closed_forms():
    check([synth.encode("ATTGCTAC"), synth.encode("GCTA"), synth.encode("CCCC"), np.zeros(0, np.uint8),
           synth.encode("TTGC")])


@pytest.mark.parametrize("seed", range(10))
def test_matrix_random(seed):
    rng = np.random.default_rng(1200 + seed)
    k = int(rng.integers(2, 21))
    alpha = int(rng.integers(1, 5))
    seqs = [rng.integers(0, alpha, size=int(rng.integers(0, 300)), dtype=np.uint8) for _ in range(k)]
    for _ in range(k):
        a, b = rng.integers(0, k, size=2)
        if a != b and seqs[a].size > 20:
            s = int(rng.integers(0, seqs[a].size - 10))
            seg = seqs[a][s:s + int(rng.integers(3, 80))]
            p = int(rng.integers(0, seqs[b].size + 1))
            seqs[b] = np.concatenate([seqs[b][:p], seg, seqs[b][p:]])
    say("matrix", seed, k)
    check(seqs)


def test_matrix_max_sequences():
    """251 sequences (the most one joined text holds): every row of best keys,
    start table and record queue in LDS is full, and some sequences are empty
    or a single base."""
    rng = np.random.default_rng(1300)
    k = 251
    seqs = [rng.integers(0, int(rng.integers(1, 5)), size=int(rng.integers(0, 24)), dtype=np.uint8)
            for _ in range(k)]
    for _ in range(60):
        a, b = rng.integers(0, k, size=2)
        if a != b and seqs[a].size > 6:
            s = int(rng.integers(0, seqs[a].size - 4))
            p = int(rng.integers(0, seqs[b].size + 1))
            seqs[b] = np.concatenate([seqs[b][:p], seqs[a][s:s + 5], seqs[b][p:]])
    seqs[7] = np.zeros(0, np.uint8)
    seqs[8] = np.array([2], np.uint8)
    check(seqs)


@pytest.mark.parametrize("lengths", [(4000, 4190), (4000, 4000, 4285), (4095,)])
def test_matrix_exact_tiles(lengths):
    """Joined lengths that are whole 4096-rank tiles (8192, 12288, 4096): no
    ragged last tile, and with one sequence no target has another to meet."""
    rng = np.random.default_rng(sum(lengths))
    seqs = [rng.integers(0, 4, size=m, dtype=np.uint8) for m in lengths]
    for i in range(1, len(seqs)):
        s = int(rng.integers(0, seqs[0].size - 300))
        seqs[i][100:300] = seqs[0][s:s + 200]
    assert (sum(lengths) + len(lengths)) % 4096 == 0
    check(seqs)


def test_matrix_noncoding():
    rng = synth.rng_for(91)
    seqs = [synth.noncoding_like(rng, int(rng.integers(1000, 20000))) for _ in range(8)]
    for i in range(1, 8):
        s = int(rng.integers(0, seqs[0].size - 600))
        seg = synth.mutate(rng, seqs[0][s:s + 500].copy(), 0.01)
        p = int(rng.integers(0, seqs[i].size))
        seqs[i] = np.concatenate([seqs[i][:p], seg, seqs[i][p:]])
    check(seqs)


def first_shared_window(a, b, L):
    """Smallest o with a[o:o+L] a substring of b (-1: none): polynomial
    hashes of every length-L window mod 2^64 as candidates, each candidate
    then compared base by base."""
    B = np.uint64(0x9E3779B97F4A7C15)
    Binv = np.uint64(pow(int(B), -1, 1 << 64))

    def windows(s):
        n = s.size - L + 1
        if n <= 0:
            return np.zeros(0, np.uint64)
        with np.errstate(over="ignore"):
            pw = np.cumprod(np.full(s.size, B, np.uint64)) * Binv        # B^j
            iw = np.cumprod(np.full(n, Binv, np.uint64)) * B             # B^-i
            pre = np.concatenate([[np.uint64(0)], np.cumsum((s.astype(np.uint64) + np.uint64(1)) * pw)])
            return (pre[L:] - pre[:n]) * iw
    hb = windows(b)
    ha = windows(a)
    if not ha.size or not hb.size:
        return -1
    for o in np.flatnonzero(np.isin(ha, hb)).tolist():
        # the hash names candidate occurrences; confirm one exactly
        if any(np.array_equal(a[o:o + L], b[q:q + L]) for q in np.flatnonzero(hb == ha[o]).tolist()):
            return o
    return -1


def test_matrix_across_chunks_and_unaligned():
    """Three noncoding-like sequences of 3M bases with shared mutated
    segments: 9M ranks span several chunks of the two-level tile scan.
    Every record (a, b) equals the oracle's overlap of a and b alone in
    length and off_p (the first offset in a whose length-L window occurs in
    b, also found by direct search), off_q holds the same substring; an
    sa/lcp pair 4 bytes off 16-byte alignment (the scalar load path) gives
    identical records."""
    rng = synth.rng_for(92)
    k = 3
    seqs = [synth.noncoding_like(rng, 3_000_000) for _ in range(k)]
    for i in range(1, k):
        for _ in range(3):
            s = int(rng.integers(0, seqs[0].size - 3000))
            seg = synth.mutate(rng, seqs[0][s:s + int(rng.integers(800, 2500))].copy(), 0.002)
            p = int(rng.integers(0, seqs[i].size))
            seqs[i] = np.concatenate([seqs[i][:p], seg, seqs[i][p:]])
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    d = torch.from_numpy(np.concatenate(seqs)).cuda()
    r = lor.longest_overlap_region(d, offs)
    n = r["sa"].numel()
    say("matrix across chunks", n)
    assert n > 2 * 4096 * 1024
    recs = lor.records_to_tuples(lor.lor_overlap_matrix(r["sa"], r["lcp"], offs))
    sa_buf = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    lcp_buf = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    sa_buf[1:].copy_(r["sa"])
    lcp_buf[1:].copy_(r["lcp"])
    assert sa_buf[1:].data_ptr() % 16 == 4
    unaligned = lor.records_to_tuples(lor.lor_overlap_matrix(sa_buf[1:], lcp_buf[1:], offs))
    assert unaligned == recs
    import oracle_pool
    ab = [(a, b) for a in range(k) for b in range(k) if a != b]
    want = dict(zip(ab, oracle_pool.pairs_overlap([(seqs[a], seqs[b]) for a, b in ab], procs=len(ab))))
    for a in range(k):
        assert recs[a * k + a] == (0, -1, -1, -1, -1)
        for b in range(k):
            if a == b:
                continue
            L, sp, op, sq, oq = recs[a * k + b]
            assert (L, op) == (want[(a, b)][0], want[(a, b)][2]), (a, b)
            assert L > 500 and (sp, sq) == (a, b)
            assert np.array_equal(seqs[a][op:op + L], seqs[b][oq:oq + L]), (a, b)
            assert op == first_shared_window(seqs[a], seqs[b], L), (a, b)
            assert recs[b * k + a][0] == L
