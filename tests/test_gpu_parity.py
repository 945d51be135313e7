"""Parity of the HIP path against the CPU oracle, element by element.

Every test calls liblor.so through its C-ABI (the ctypes binding) on cuda:0
and compares with the oracle on the same seeded inputs. Integers only, so
every comparison is exact.
"""
import itertools
import sys

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1404_3448_amd import lor, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ------------------------------------------------------------ radix sort

def _keys_u32(rng, n, mode):
    if mode == "wide":
        return rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    if mode == "dups":
        return (rng.integers(0, 7, size=n).astype(np.uint32) * np.uint32(0x01010101))
    return rng.integers(0, 300, size=n).astype(np.uint32) << np.uint32(rng.integers(0, 20))


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1000, 4095, 4096, 4097, 262147, 1 << 20, (1 << 22) + 12345])
@pytest.mark.parametrize("bits", [(0, 32), (0, 8), (3, 17), (0, 15)])
@pytest.mark.parametrize("mode", ["wide", "dups", "skew"])
def test_sort_pairs_u32(n, bits, mode):
    say("sort u32", n, bits, mode)
    rng = np.random.default_rng(n * 7 + bits[0])
    keys = _keys_u32(rng, n, mode)
    vals = rng.permutation(n).astype(np.int32)
    lo, hi = bits
    digit = (keys.astype(np.uint64) >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1)
    order = np.argsort(digit, kind="stable")
    k = dev(keys.view(np.int32))
    v = dev(vals)
    lor.lor_sort_pairs_u32(k, v, lo, hi)
    assert np.array_equal(host(k).view(np.uint32), keys[order])
    assert np.array_equal(host(v), vals[order])


@pytest.mark.parametrize("n", [1, 100, 3073, 200001, (1 << 21) + 77])
@pytest.mark.parametrize("bits", [(0, 64), (5, 45), (0, 21)])
def test_sort_pairs_u64(n, bits):
    say("sort u64", n, bits)
    rng = np.random.default_rng(n + bits[1])
    keys = rng.integers(0, 1 << 63, size=n, dtype=np.uint64) | (rng.integers(0, 2, size=n, dtype=np.uint64) << np.uint64(63))
    keys[rng.random(n) < 0.3] = keys[0]
    vals = np.arange(n, dtype=np.int32)
    lo, hi = bits
    mask = np.uint64((1 << (hi - lo)) - 1) if hi - lo < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    digit = (keys >> np.uint64(lo)) & mask
    order = np.argsort(digit, kind="stable")
    k = dev(keys.view(np.int64))
    v = dev(vals)
    lor.lor_sort_pairs_u64(k, v, lo, hi)
    assert np.array_equal(host(k).view(np.uint64), keys[order])
    assert np.array_equal(host(v), vals[order])


def test_sort_pairs_split_example(golden):
    """One 1-bit pass reproduces the split example of Section IV."""
    g = golden["paper_examples"]["split_example"]
    k = dev(np.array(g["keys"], dtype=np.int32))
    v = dev(np.arange(5, dtype=np.int32))
    lor.lor_sort_pairs_u32(k, v, g["bit"], g["bit"] + 1)
    assert list(host(k)) == g["out"]
    dest = np.empty(5, dtype=np.int64)
    dest[host(v)] = np.arange(5)
    assert list(dest) == g["dest"]


# ------------------------------------------------------------- DC3 core

def sa_i32(text, alphabet):
    return host(lor.lor_suffix_array_i32(dev(np.asarray(text, dtype=np.int32)), alphabet))


def test_dc3_paper_table1(golden):
    g = golden["paper_examples"]
    t = [{"A": 1, "C": 2, "G": 3, "T": 4}[c] for c in g["text"]]
    assert list(sa_i32(t, 4)) == g["table1_sa"]["value"]


def test_dc3_all_short_binary_texts():
    for n in range(1, 9):
        for t in itertools.product([1, 2], repeat=n):
            assert list(sa_i32(t, 2)) == brute.suffix_array(list(t)), t


@pytest.mark.parametrize("alphabet", [1, 2, 4, 255, 4096, (1 << 20) + 1, (1 << 30) + 7])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 97, 1000, 4099, 70001])
def test_dc3_random_texts(alphabet, n):
    say("dc3", alphabet, n)
    rng = np.random.default_rng(alphabet * 31 + n)
    t = rng.integers(1, alphabet + 1, size=n).astype(np.int32)
    assert np.array_equal(sa_i32(t, alphabet), oracle.suffix_array(t))


@pytest.mark.parametrize("period", [1, 2, 3, 5, 7, 12])
@pytest.mark.parametrize("n", [10, 999, 30001])
def test_dc3_periodic_texts(period, n):
    """Long repeats force deep recursion (A^n recurses about log_1.5 n times)."""
    say("dc3 periodic", period, n)
    rng = np.random.default_rng(period * 1000 + n)
    unit = rng.integers(1, 4, size=period).astype(np.int32)
    t = np.resize(unit, n)
    if n > 100:
        hit = rng.integers(0, n, size=3)
        t[hit] = 4
    assert np.array_equal(sa_i32(t, 4), oracle.suffix_array(t))


@pytest.mark.parametrize("offset", [0, 1, 2, 3])
@pytest.mark.parametrize("alphabet", [4, 40])
def test_dc3_text_at_any_alignment(offset, alphabet):
    """A text that starts 4, 8 or 12 bytes past a 16-byte boundary takes the
    per-symbol naming path (the word-window path needs 16-byte alignment);
    both must give the oracle's order."""
    n = 50_000
    say("dc3 offset", offset, alphabet)
    rng = np.random.default_rng(77 + offset + alphabet)
    t = rng.integers(1, alphabet + 1, size=n).astype(np.int32)
    buf = torch.zeros(n + 8, dtype=torch.int32, device="cuda")
    view = buf[offset:offset + n]
    view.copy_(torch.from_numpy(t))
    assert view.data_ptr() % 16 == 4 * offset
    got = host(lor.lor_suffix_array_i32(view, alphabet))
    assert np.array_equal(got, oracle.suffix_array(t))


# ----------------------------------------------------------- joined text

def build(seqs):
    seqs = [np.asarray(s, dtype=np.uint8) for s in seqs]
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    cat = np.concatenate(seqs) if sum(s.size for s in seqs) else np.zeros(1, np.uint8)
    return dev(cat), offs


def test_build_sa_joined_example(golden):
    g = golden["paper_examples"]
    seqs, offs = build([synth.encode(g["text"])])
    sa, joined = lor.lor_build_sa(seqs, offs)
    assert list(host(joined)) == list(synth.encode(g["text"])) + [4]
    assert list(host(sa)) == g["joined_example"]["sa"]
    lcp, isa = lor.lor_build_lcp(joined, sa, want_isa=True)
    assert list(host(lcp)) == g["joined_example"]["lcp"]
    assert list(host(isa)) == list(oracle.isa(np.array(g["joined_example"]["sa"], np.int32)))


@pytest.mark.parametrize("seed", range(16))
def test_build_sa_lcp_many_sequences(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 9)) if seed < 12 else int(rng.integers(100, 252))
    alpha = int(rng.integers(1, 5))
    seqs = [rng.integers(0, alpha, size=int(rng.integers(0, 3000)), dtype=np.uint8) for _ in range(k)]
    if seed % 4 == 0:
        seqs[0] = np.zeros(0, np.uint8)
    say("build_sa", seed, k, [s.size for s in seqs][:8])
    d, offs = build(seqs)
    sa, joined = lor.lor_build_sa(d, offs)
    want_joined = oracle.join(np.concatenate(seqs), offs)
    assert np.array_equal(host(joined), want_joined)
    want_sa = oracle.suffix_array(want_joined)
    assert np.array_equal(host(sa), want_sa)
    lcp, isa = lor.lor_build_lcp(joined, sa, want_isa=True)
    assert np.array_equal(host(lcp), oracle.lcp(want_joined, want_sa))
    assert np.array_equal(host(isa), oracle.isa(want_sa))
    ov = lor.lor_longest_overlap(sa, lcp, offs)
    assert ov == oracle.overlap(want_sa, oracle.lcp(want_joined, want_sa), offs)


@pytest.mark.parametrize("shift", [0, 1, 3, 7, 13])
def test_join_from_misaligned_bases_and_bad_base_inside(shift):
    """The bases start `shift` bytes into their buffer, so the join's word
    loads meet every byte alignment; a bad base deep inside a long sequence
    (a window copied whole) is still reported."""
    rng = np.random.default_rng(40 + shift)
    seqs = [rng.integers(0, 4, size=n, dtype=np.uint8) for n in (5003, 17, 0, 4096, 2999)]
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    flat = np.concatenate(seqs)
    buf = torch.zeros(flat.size + shift + 16, dtype=torch.uint8, device="cuda")
    buf[shift:shift + flat.size].copy_(torch.from_numpy(flat))
    d = buf[shift:shift + flat.size]
    sa, joined = lor.lor_build_sa(d, offs)
    want = oracle.join(flat, offs)
    assert np.array_equal(host(joined), want)
    assert np.array_equal(host(sa), oracle.suffix_array(want))
    bad = flat.copy()
    bad[2500] = 7
    buf[shift:shift + flat.size].copy_(torch.from_numpy(bad))
    with pytest.raises(lor.LorError) as e:
        lor.lor_build_sa(d, offs)
    assert e.value.status == lor.LOR_EALPHABET


def test_build_sa_rejects_bad_base():
    d, offs = build([[0, 1, 2], [3, 7, 1]])
    with pytest.raises(lor.LorError) as e:
        lor.lor_build_sa(d, offs)
    assert e.value.status == lor.LOR_EALPHABET


def test_lor_check_reads_the_workspace_header():
    """lor_check returns what the device left in a call's workspace header:
    nothing after a good call, the bad base after a bad one."""
    good, goff = build([[0, 1, 2, 3], [3, 2, 1]])
    bad, boff = build([[0, 1, 2], [3, 7, 1]])
    ws = torch.empty(lor.lor_build_sa_workspace(8, 2), dtype=torch.uint8, device="cuda")
    lor.lor_build_sa(good, goff, ws=ws)
    assert lor.lor_check(ws) == lor.LOR_OK
    with pytest.raises(lor.LorError):
        lor.lor_build_sa(bad, boff, ws=ws)
    assert lor.lor_check(ws) == lor.LOR_EALPHABET
    lor.lor_build_sa(good, goff, ws=ws)   # every call clears the header first
    assert lor.lor_check(ws) == lor.LOR_OK


def test_repeated_calls_are_bit_identical():
    w = synth.noncoding_pair(seed=21, n=300_000, segments=4)
    d, offs = dev(w.concat), w.offsets
    sa1, j1 = lor.lor_build_sa(d, offs)
    l1, _ = lor.lor_build_lcp(j1, sa1)
    first = (host(sa1).copy(), host(l1).copy())
    for _ in range(2):
        sa2, j2 = lor.lor_build_sa(d, offs)
        l2, _ = lor.lor_build_lcp(j2, sa2)
        assert np.array_equal(host(sa2), first[0]) and np.array_equal(host(l2), first[1])


# --------------------------------------------------------------- overlap

@pytest.mark.parametrize("case", range(8))
def test_overlap_closed_forms(golden, case):
    c = golden["overlap_closed_forms"]["cases"][case]
    d, offs = build([synth.encode(c["a"]), synth.encode(c["b"])])
    r = lor.longest_overlap_region(d, offs)
    assert list(r["overlap"]) == c["expect"]


@pytest.mark.parametrize("seed", range(12))
def test_overlap_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    k = int(rng.integers(2, 5))
    alpha = int(rng.integers(1, 5))
    seqs = [rng.integers(0, alpha, size=int(rng.integers(0, 30)), dtype=np.uint8) for _ in range(k)]
    d, offs = build(seqs)
    r = lor.longest_overlap_region(d, offs)
    assert r["overlap"] == brute.longest_overlap(seqs)


def test_tiny_pair_workload():
    """50k + 50k uniform bases with a planted 500-base copy: SA, LCP and the
    overlap equal the oracle's; the overlap equals the O(nm) DP's."""
    w = synth.tiny_pair()
    d = dev(w.concat)
    r = lor.longest_overlap_region(d, w.offsets, want_isa=True)
    joined = oracle.join(w.concat, w.offsets)
    want_sa = oracle.suffix_array(joined)
    want_lcp = oracle.lcp(joined, want_sa)
    assert np.array_equal(host(r["joined"]), joined)
    assert np.array_equal(host(r["sa"]), want_sa)
    assert np.array_equal(host(r["lcp"]), want_lcp)
    L, sp, op, sq, oq = r["overlap"]
    assert r["overlap"] == oracle.overlap(want_sa, want_lcp, w.offsets)
    assert (L, op, oq) == oracle.lcs_dp(w.seqs[0], w.seqs[1])
    assert L >= 500


# ------------------------------------------------------------------- RMQ

@pytest.mark.parametrize("n_bases", [3, 17, 1000, 40000])
@pytest.mark.parametrize("compact", [False, True])
def test_rmq_range_and_pair_queries(n_bases, compact):
    rng = np.random.default_rng(n_bases)
    w = synth.noncoding_pair(seed=n_bases, n=n_bases, segments=2, seg_lo=2, seg_hi=max(3, n_bases // 3))
    d = dev(w.concat)
    r = lor.longest_overlap_region(d, w.offsets, want_isa=True)
    joined = oracle.join(w.concat, w.offsets)
    n = joined.size
    lcp_h = host(r["lcp"])
    if compact:
        rmq = lor.lor_rmq_compact_build(r["lcp"])
        nb = -(-n // 64)
        assert rmq.compact and rmq.levels == (nb.bit_length() - 1 if nb >= 2 else 0)
    else:
        rmq = lor.lor_rmq_build(r["lcp"])
        assert rmq.levels == n.bit_length() - 1
    lo = rng.integers(0, n, size=3000)
    hi = np.minimum(n - 1, lo + rng.integers(0, n, size=3000) % (1 + rng.integers(1, n + 1, size=3000)))
    mn, am = lor.lor_rmq_query(rmq, r["lcp"], r["isa"], 0, dev(lo.astype(np.int32)), dev(hi.astype(np.int32)),
                               want_argmin=True)
    mn, am = host(mn), host(am)
    for k in range(lo.size):
        assert (mn[k], am[k]) == oracle.range_min(lcp_h, lo[k], hi[k])
    qi = rng.integers(0, n, size=5000).astype(np.int32)
    qj = rng.integers(0, n, size=5000).astype(np.int32)
    qj[:50] = qi[:50]
    got, _ = lor.lor_rmq_query(rmq, r["lcp"], r["isa"], 1, dev(qi), dev(qj))
    assert np.array_equal(host(got), oracle.pair_queries(joined, qi, qj))
    bad_i = np.array([-1, n, 0, 5 % n], dtype=np.int32)
    bad_j = np.array([0, 0, n + 3, -7], dtype=np.int32)
    got, am = lor.lor_rmq_query(rmq, r["lcp"], r["isa"], 1, dev(bad_i), dev(bad_j), want_argmin=True)
    assert list(host(got)) == [-1] * 4 and list(host(am)) == [-1] * 4
    got, _ = lor.lor_rmq_query(rmq, r["lcp"], r["isa"], 0, dev(np.array([3 % n], np.int32)),
                               dev(np.array([0], np.int32)))
    assert list(host(got)) == ([-1] if 3 % n > 0 else [0])


# ------------------------------------------------------- larger workloads

_TRACE_CHILD = """
import sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_1404_3448_amd import lor, synth
w = synth.long_text(seed=int(sys.argv[2]), num_seqs=2, seq_len=int(sys.argv[3]), num_queries=1)
lor.lor_build_sa(torch.from_numpy(w.concat).cuda(), w.offsets)
torch.cuda.synchronize()
"""


@pytest.mark.parametrize("seed", [31, 32])
def test_deep_levels_from_parent_order(seed):
    """Noncoding-like text with tandem repeats (2 x 2^21 bases): its deep DC3
    levels take the parent-order path (first-symbol order from the parent
    level, merge records only for repeating first symbols), as the level trace
    of the same call in a child process shows; SA and LCP equal the oracle's."""
    import os
    import subprocess
    seq_len = 1 << 21
    env = dict(os.environ, LOR_TRACE="1")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("parent-order trace child", seed)
    tr = subprocess.run([sys.executable, "-c", _TRACE_CHILD, root, str(seed), str(seq_len)], env=env,
                        capture_output=True, text=True, timeout=300)
    assert tr.returncode == 0, tr.stderr[-2000:]
    assert tr.stderr.count("parent-order") >= 2, tr.stderr[-2000:]
    w = synth.long_text(seed=seed, num_seqs=2, seq_len=seq_len, num_queries=1)
    r = lor.longest_overlap_region(dev(w.concat), w.offsets)
    joined = oracle.join(w.concat, w.offsets)
    want_sa = oracle.suffix_array(joined)
    assert np.array_equal(host(r["sa"]), want_sa)
    assert np.array_equal(host(r["lcp"]), oracle.lcp(joined, want_sa))

def test_noncoding_pair_8m():
    """The 8M + 8M workload at full size: SA and LCP equal the oracle's
    (comparison sort + direct LCP), and so does the overlap."""
    w = synth.noncoding_pair()
    say("8M+8M generated")
    d = dev(w.concat)
    r = lor.longest_overlap_region(d, w.offsets)
    joined = oracle.join(w.concat, w.offsets)
    want_sa = oracle.suffix_array(joined)
    want_lcp = oracle.lcp(joined, want_sa)
    say("8M+8M oracle done")
    assert np.array_equal(host(r["sa"]), want_sa)
    assert np.array_equal(host(r["lcp"]), want_lcp)
    assert r["overlap"] == oracle.overlap(want_sa, want_lcp, w.offsets)


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_long_text_1g_full_size():
    """The 1G-base workload (16 x 2^26 bases, 10M queries) at full size, in the
    benchmark's launch configuration. SA and LCP are certified by the oracle's
    certificate (permutation + strict adjacent order + exact LCP, which proves
    them equal to the oracle's definition); ISA is checked as the inverse of SA;
    the overlap equals the oracle's scan of the certified arrays; 20,000 sampled
    suffix-pair queries equal direct character comparison."""
    w = synth.long_text()
    n = w.joined_length
    say("1G generated", n)
    seqs = dev(w.concat)
    joined = torch.empty(n, dtype=torch.uint8, device=DEV)
    sa = torch.empty(n, dtype=torch.int32, device=DEV)
    lcp = torch.empty(n, dtype=torch.int32, device=DEV)
    isa = torch.empty(n, dtype=torch.int32, device=DEV)
    lor.lor_build_sa(seqs, w.offsets, joined_out=joined, sa_out=sa)
    lor.lor_build_lcp(joined, sa, lcp_out=lcp, isa_out=isa)
    rmq = lor.lor_rmq_build(lcp)
    qi, qj = dev(w.queries[0]), dev(w.queries[1])
    got, _ = lor.lor_rmq_query(rmq, lcp, isa, 1, qi, qj)
    ov = lor.lor_longest_overlap(sa, lcp, w.offsets)
    got_h = host(got)
    del rmq, qi, qj, got, seqs
    joined_h, sa_h, lcp_h, isa_h = host(joined), host(sa), host(lcp), host(isa)
    del joined, sa, lcp, isa
    torch.cuda.empty_cache()
    say("1G GPU path done, certifying on the host")
    assert np.array_equal(joined_h, oracle.join(w.concat, w.offsets))
    assert oracle.certify(joined_h, sa_h, lcp_h) == -1
    assert np.array_equal(isa_h[sa_h], np.arange(n, dtype=np.int32))
    assert ov == oracle.overlap(sa_h, lcp_h, w.offsets)
    rng = np.random.default_rng(33)
    pick = rng.choice(w.queries[0].size, size=20000, replace=False)
    want = oracle.pair_queries(joined_h, w.queries[0][pick], w.queries[1][pick])
    assert np.array_equal(got_h[pick], want)


@pytest.mark.parametrize("top", [65535, 65536, 3_000_000])
def test_rmq_table_width_boundary(top):
    """Levels are stored as 16-bit entries only when the largest LCP value is
    at most 65535: at 65535 (16-bit), 65536 and 3M (32-bit) every level of
    an 18-level table (fused, chained and single-level passes) answers as
    the plain minimum does, with the leftmost position."""
    n = 300_007
    say("rmq width", top)
    rng = np.random.default_rng(top)
    lcp_h = rng.integers(0, 70000, size=n).astype(np.int64)
    lcp_h = np.minimum(lcp_h, top).astype(np.int32)
    lcp_h[rng.integers(0, n)] = top
    lcp = dev(lcp_h)
    rmq = lor.lor_rmq_build(lcp)
    lo = rng.integers(0, n, size=6000)
    span = np.where(rng.random(6000) < 0.5, rng.integers(0, 5000, size=6000), rng.integers(0, n, size=6000))
    hi = np.minimum(n - 1, lo + span)
    m, a = lor.lor_rmq_query(rmq, lcp, None, 0, dev(lo.astype(np.int32)), dev(hi.astype(np.int32)),
                             want_argmin=True)
    m, a = host(m), host(a)
    for k in range(0, lo.size, 3):
        assert (m[k], a[k]) == oracle.range_min(lcp_h, lo[k], hi[k]), k
    whole = lor.lor_rmq_query(rmq, lcp, None, 0, dev(np.array([0], np.int32)),
                              dev(np.array([n - 1], np.int32)), want_argmin=True)
    assert (host(whole[0])[0], host(whole[1])[0]) == oracle.range_min(lcp_h, 0, n - 1)


@pytest.mark.parametrize("n", [1500, 2049, 4095, 5000, 9000, 20000, 33000])
@pytest.mark.parametrize("top", [1000, 100000])
def test_rmq_every_level_count(n, top):
    """Tables of 10 to 15 levels in 16- and 32-bit entries: the level passes
    above the register pass take three levels at a time, so these sizes end
    with a pass of one, two or three levels. For every level k, ranges of
    exactly 2^k entries and of 2^k + 1 .. 2^(k+1) - 1 entries, at random
    starts and flush with both ends, answer as the plain minimum does, with
    the leftmost position; smooth values with noise make ties rare and every
    window's minimum depend on where it lies."""
    say("rmq levels", n, top)
    rng = np.random.default_rng(n + top)
    x = np.arange(n)
    lcp_h = (top / 2 + top / 3 * np.sin(x / 97.0) + rng.integers(0, max(2, top // 50), size=n)).astype(np.int32)
    lcp_h[rng.integers(0, n)] = top
    lcp = dev(lcp_h)
    rmq = lor.lor_rmq_build(lcp)
    levels = n.bit_length() - 1
    assert rmq.levels == levels
    lo, hi = [], []
    for k in range(levels + 1):
        w = 1 << k
        for span in (w, min(n, w + 1 + int(rng.integers(0, w))), min(n, 2 * w - 1)):
            for start in (0, n - span, *rng.integers(0, n - span + 1, size=6)):
                lo.append(int(start))
                hi.append(int(start) + span - 1)
    lo, hi = np.array(lo), np.array(hi)
    m, a = lor.lor_rmq_query(rmq, lcp, None, 0, dev(lo.astype(np.int32)), dev(hi.astype(np.int32)),
                             want_argmin=True)
    m, a = host(m), host(a)
    for q in range(lo.size):
        assert (m[q], a[q]) == oracle.range_min(lcp_h, lo[q], hi[q]), (q, lo[q], hi[q])


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 128, 129, 191, 1000, 4097, 100003])
@pytest.mark.parametrize("values", [2, 50, 1 << 20])
def test_rmq_compact_equals_oracle_and_full_table(n, values):
    """Compact (block) table: values and leftmost positions equal the plain
    minimum and the full table's, for ranges inside a block, across a block
    boundary and spanning many blocks; few distinct values make ties common."""
    say("rmq compact", n, values)
    rng = np.random.default_rng(n * 31 + values)
    lcp_h = rng.integers(0, values, size=n).astype(np.int32)
    lcp = dev(lcp_h)
    full = lor.lor_rmq_build(lcp) if n >= 1 else None
    comp = lor.lor_rmq_compact_build(lcp)
    lo = rng.integers(0, n, size=4000)
    span = np.where(rng.random(4000) < 0.5, rng.integers(0, 130, size=4000), rng.integers(0, n, size=4000))
    hi = np.minimum(n - 1, lo + span)
    lo_d, hi_d = dev(lo.astype(np.int32)), dev(hi.astype(np.int32))
    mc, ac = lor.lor_rmq_query(comp, lcp, None, 0, lo_d, hi_d, want_argmin=True)
    mf, af = lor.lor_rmq_query(full, lcp, None, 0, lo_d, hi_d, want_argmin=True)
    mc, ac, mf, af = host(mc), host(ac), host(mf), host(af)
    assert np.array_equal(mc, mf) and np.array_equal(ac, af)
    for k in range(0, lo.size, 7):
        assert (mc[k], ac[k]) == oracle.range_min(lcp_h, lo[k], hi[k])


def test_kernel_timing_registry_and_filter():
    """Event timing counts every launch of every family; limited to one
    family it records that family alone, with the same launch count."""
    rng = np.random.default_rng(8)
    seqs = [rng.integers(0, 4, size=5000, dtype=np.uint8) for _ in range(3)]
    offs = np.concatenate([[0], np.cumsum([s.size for s in seqs])]).astype(np.int64)
    d = torch.from_numpy(np.concatenate(seqs)).cuda()
    try:
        lor.lor_timing_only(None)
        lor.lor_timing_reset()
        lor.lor_timing_enable(True)
        lor.longest_overlap_region(d, offs)
        torch.cuda.synchronize()
        everything = lor.lor_timing_read()
        assert {"k_join", "k_radix_scatter", "k_merge", "k_plcp"} <= set(everything)
        assert all(v["launches"] > 0 and v["ms"] > 0 for v in everything.values())
        lor.lor_timing_reset()
        lor.lor_timing_only("k_radix_scatter")
        lor.longest_overlap_region(d, offs)
        torch.cuda.synchronize()
        one = lor.lor_timing_read()
        assert set(one) == {"k_radix_scatter"}
        assert one["k_radix_scatter"]["launches"] == everything["k_radix_scatter"]["launches"]
    finally:
        lor.lor_timing_enable(False)
        lor.lor_timing_only(None)
        lor.lor_timing_reset()
