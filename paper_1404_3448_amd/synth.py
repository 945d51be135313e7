"""Seeded synthetic DNA inputs for the longest-overlap-region path.

This module only draws random sequences and queries. It holds none of the
method's arithmetic (no suffix sorting, no LCP, no overlap scan), imports
nothing else from this package, and serves both the CPU oracle tests and the
GPU path's tests and benchmark.

The paper measures on three NCBI non-coding records (Section V). They are not
available here; the generators below stand in for them with non-coding-like
synthetic text: a base composition of 40% GC, tandem repeats covering about a
tenth of each sequence, and shared segments planted between the two members of
a pair (with point mutations for the long workloads).

Symbols are uint8 codes A=0, C=1, G=2, T=3. Every generator is a pure function
of its seed: numpy ``Generator(PCG64(seed))``, applied per sequence in the
order base text -> tandem repeats -> planted segments.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

A, C, G, T = 0, 1, 2, 3

# 40% GC: P(A) = P(T) = 0.3, P(C) = P(G) = 0.2, drawn as a uniform digit 0..9.
_GC40_LUT = np.array([A, A, A, C, C, G, G, T, T, T], dtype=np.uint8)


def rng_for(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_bases(rng: np.random.Generator, n: int) -> np.ndarray:
    """iid uniform over {A,C,G,T}."""
    return rng.integers(0, 4, size=n, dtype=np.uint8)


def gc40_bases(rng: np.random.Generator, n: int, chunk: int = 1 << 24) -> np.ndarray:
    """iid bases with 40% GC content, drawn in chunks to bound host memory."""
    out = np.empty(n, dtype=np.uint8)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = _GC40_LUT[rng.integers(0, 10, size=e - s, dtype=np.uint8)]
    return out


def add_tandem_repeats(rng: np.random.Generator, seq: np.ndarray, coverage: float = 0.10) -> None:
    """Overwrite tandem repeats at uniform positions until >= coverage of the
    positions lie inside at least one repeat. Each repeat has a period drawn
    uniformly from 2..6, a unit drawn iid with 40% GC, and 10..200 copies."""
    n = seq.size
    if n == 0:
        return
    covered = np.zeros(n, dtype=bool)
    need = int(math.ceil(coverage * n))
    have = 0
    while have < need:
        pos = int(rng.integers(0, n))
        period = int(rng.integers(2, 7))
        copies = int(rng.integers(10, 201))
        unit = _GC40_LUT[rng.integers(0, 10, size=period, dtype=np.uint8)]
        length = min(period * copies, n - pos)
        seq[pos:pos + length] = np.tile(unit, copies)[:length]
        have += length - int(np.count_nonzero(covered[pos:pos + length]))
        covered[pos:pos + length] = True


def noncoding_like(rng: np.random.Generator, n: int) -> np.ndarray:
    """40% GC base text plus tandem repeats covering about 10% of it."""
    s = gc40_bases(rng, n)
    add_tandem_repeats(rng, s)
    return s


def mutate(rng: np.random.Generator, seg: np.ndarray, p: float) -> np.ndarray:
    """Substitute each base with probability p by a uniformly chosen different base."""
    seg = seg.copy()
    hit = rng.random(seg.size) < p
    k = int(np.count_nonzero(hit))
    if k:
        shift = rng.integers(1, 4, size=k, dtype=np.uint8)
        seg[hit] = (seg[hit] + shift) % 4
    return seg


def plant(rng: np.random.Generator, a: np.ndarray, b: np.ndarray, length: int, p_mut: float = 0.0):
    """Copy a segment of `length` bases from a uniform position of a to a
    uniform position of b (in place), optionally point-mutated.
    Returns (pos_a, pos_b)."""
    length = min(length, a.size, b.size)
    pa = int(rng.integers(0, a.size - length + 1))
    pb = int(rng.integers(0, b.size - length + 1))
    seg = a[pa:pa + length]
    if p_mut > 0:
        seg = mutate(rng, seg, p_mut)
    b[pb:pb + length] = seg
    return pa, pb


@dataclass
class Workload:
    name: str
    seqs: list                       # list of uint8 arrays (codes 0..3)
    planted: list = field(default_factory=list)   # (pos_a, pos_b, length) for planted copies
    queries: tuple | None = None     # (qi, qj) int32 arrays of joined positions

    @property
    def offsets(self) -> np.ndarray:
        """int64 offsets[k+1] of the sequences inside the separator-free concatenation."""
        return np.concatenate([[0], np.cumsum([s.size for s in self.seqs])]).astype(np.int64)

    @property
    def concat(self) -> np.ndarray:
        return np.concatenate(self.seqs) if self.seqs else np.zeros(0, np.uint8)

    @property
    def joined_length(self) -> int:
        return int(sum(s.size for s in self.seqs)) + len(self.seqs)


def tiny_pair(seed: int = 1, n: int = 50_000, planted_len: int = 500) -> Workload:
    """Two iid uniform sequences of n bases with one exact planted copy of
    planted_len bases from A to B (the 50k + 50k workload)."""
    rng = rng_for(seed)
    a = uniform_bases(rng, n)
    b = uniform_bases(rng, n)
    pa, pb = plant(rng, a, b, planted_len)
    return Workload(f"pair-{n}+{n}-planted{planted_len}", [a, b], [(pa, pb, planted_len)])


def noncoding_pair(seed: int = 2, n: int = 1 << 23, segments: int = 20,
                   seg_lo: float = 1e3, seg_hi: float = 1e4, p_mut: float = 0.01) -> Workload:
    """One pair of n + n noncoding-like bases with `segments` planted shared
    segments of log-uniform length in [seg_lo, seg_hi], each base mutated with
    probability p_mut (the 8M + 8M workload at the defaults)."""
    rng = rng_for(seed)
    a = noncoding_like(rng, n)
    b = noncoding_like(rng, n)
    planted = []
    for _ in range(segments):
        length = int(round(math.exp(rng.uniform(math.log(seg_lo), math.log(seg_hi)))))
        length = max(1, min(length, max(1, min(a.size, b.size) // 4)))
        pa, pb = plant(rng, a, b, length, p_mut)
        planted.append((pa, pb, length))
    return Workload(f"pair-{n}+{n}-noncoding", [a, b], planted)


def long_text(seed: int = 3, num_seqs: int = 16, seq_len: int = 1 << 26,
              num_queries: int = 10_000_000) -> Workload:
    """num_seqs noncoding-like sequences of seq_len bases each (no planted
    segments) and num_queries iid uniform suffix-pair queries over the joined
    text (the 1G-base workload at the defaults: 16 x 67,108,864 bases,
    joined length 1,073,741,840, 10M queries)."""
    data_ss, query_ss = np.random.SeedSequence(seed).spawn(2)
    rng = np.random.Generator(np.random.PCG64(data_ss))
    seqs = [noncoding_like(rng, seq_len) for _ in range(num_seqs)]
    n = num_seqs * seq_len + num_seqs
    qrng = np.random.Generator(np.random.PCG64(query_ss))
    qi = qrng.integers(0, n, size=num_queries, dtype=np.int64).astype(np.int32)
    qj = qrng.integers(0, n, size=num_queries, dtype=np.int64).astype(np.int32)
    return Workload(f"text-{num_seqs}x{seq_len}", seqs, [], (qi, qj))


def batched_pairs(seed: int = 4, num_pairs: int = 4096, lo: float = 1e3, hi: float = 1e6) -> list:
    """num_pairs independent noncoding-like pairs. The pair's total length is
    log-uniform in [lo, hi], split |A| = floor(L/2), |B| = L - |A|. Each pair
    gets min(20, max(1, min(|A|,|B|) // 40000)) planted segments, each with a
    log-uniform length in [1e3, 1e4] clipped to min(|A|,|B|) // 4, mutated at
    1%. Sub-seeds come from SeedSequence(seed).spawn(num_pairs)."""
    out = []
    for p, ss in enumerate(np.random.SeedSequence(seed).spawn(num_pairs)):
        rng = np.random.Generator(np.random.PCG64(ss))
        total = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        na = total // 2
        nb = total - na
        a = noncoding_like(rng, na)
        b = noncoding_like(rng, nb)
        planted = []
        m = min(na, nb)
        for _ in range(min(20, max(1, m // 40000))):
            length = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e4)))))
            length = max(1, min(length, max(1, m // 4)))
            pa, pb = plant(rng, a, b, length, 0.01)
            planted.append((pa, pb, length))
        out.append(Workload(f"batch{p}", [a, b], planted))
    return out


def ref_queries(seed: int = 6, ref_len: int = 1 << 22, num_queries: int = 1 << 16, lo: float = 100,
                hi: float = 2000) -> Workload:
    """One noncoding-like reference and many noncoding-like queries (the
    shape of Section V: a reference group against many query sequences).
    Query lengths are log-uniform in [lo, hi]; every third query carries a
    segment copied from the reference (length log-uniform in [20, q/2],
    1% point mutations) at a uniform position. seqs[0] is the reference."""
    rng = rng_for(seed)
    ref = noncoding_like(rng, ref_len)
    seqs = [ref]
    planted = []
    for i in range(num_queries):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        q = noncoding_like(rng, n)
        if i % 3 == 0 and n >= 40:
            length = int(round(math.exp(rng.uniform(math.log(20), math.log(n / 2)))))
            s = int(rng.integers(0, ref_len - length))
            p = int(rng.integers(0, n - length + 1))
            q[p:p + length] = mutate(rng, ref[s:s + length].copy(), 0.01)
            planted.append((i + 1, p, s, length))
        seqs.append(q)
    return Workload("ref_queries", seqs, planted)


def random_text(seed: int, n: int, alphabet: int = 4) -> np.ndarray:
    """iid uniform codes in [0, alphabet) for small test cases."""
    return rng_for(seed).integers(0, alphabet, size=n, dtype=np.uint8)


def encode(s: str) -> np.ndarray:
    """'ACGT' string -> uint8 codes."""
    lut = {"A": A, "C": C, "G": G, "T": T}
    return np.array([lut[ch] for ch in s], dtype=np.uint8)
