"""Pure-Python brute force for tiny inputs (test infrastructure only).

Every function here enumerates its answer from the definition with Python's
own sequence comparison and slicing; nothing is shared with the C oracle or
the GPU path.
"""
from __future__ import annotations


def suffix_array(text) -> list:
    """Sort the suffixes of text as Python lists; a proper prefix is smaller."""
    t = list(text)
    return sorted(range(len(t)), key=lambda i: t[i:])


def lcp_pair(text, i: int, j: int) -> int:
    t = list(text)
    h = 0
    while i + h < len(t) and j + h < len(t) and t[i + h] == t[j + h]:
        h += 1
    return h


def lcp_array(text, sa) -> list:
    return [0] + [lcp_pair(text, sa[r - 1], sa[r]) for r in range(1, len(sa))]


def joined(seqs) -> list:
    out = []
    for j, s in enumerate(seqs):
        out.extend(int(x) for x in s)
        out.append(4 + j)
    return out


def longest_overlap(seqs) -> tuple:
    """Longest substring shared by two different sequences, by enumerating
    every pair of start positions in every pair of sequences. Among all
    maximal-length occurrences the pair of joined positions (p, q), p < q, that
    is lexicographically smallest is reported as
    (L, seq_p, off_p, seq_q, off_q); L == 0 gives -1 for the rest."""
    seqs = [list(int(x) for x in s) for s in seqs]
    starts = []
    base = 0
    for j, s in enumerate(seqs):
        starts.append(base)
        base += len(s) + 1
    best = (0, None, None)
    for a in range(len(seqs)):
        for b in range(a + 1, len(seqs)):
            sa_, sb_ = seqs[a], seqs[b]
            for x in range(len(sa_)):
                for y in range(len(sb_)):
                    h = 0
                    while x + h < len(sa_) and y + h < len(sb_) and sa_[x + h] == sb_[y + h]:
                        h += 1
                    if h == 0:
                        continue
                    p, q = starts[a] + x, starts[b] + y
                    cand = (h, -p, -q)
                    if best[0] == 0 or cand > (best[0], -best[1], -best[2]):
                        best = (h, p, q)
    if best[0] == 0:
        return (0, -1, -1, -1, -1)
    L, p, q = best

    def locate(pos):
        for j in range(len(seqs) - 1, -1, -1):
            if pos >= starts[j]:
                return j, pos - starts[j]
        raise AssertionError

    sp, op = locate(p)
    sq, oq = locate(q)
    return (L, sp, op, sq, oq)


def range_min(a, lo: int, hi: int) -> tuple:
    seg = list(a[lo:hi + 1])
    v = min(seg)
    return v, lo + seg.index(v)


def split_by_bit(keys, bit: int) -> dict:
    """One split step of a binary radix sort (Section IV): L holds the tested
    bit of every key, E its complement, F the exclusive prefix sum of E,
    totalFalse = E[n-1] + F[n-1] the number of zero bits; a key with bit 0 goes
    to F[i], a key with bit 1 to i - F[i] + totalFalse. The output lists the
    keys at their destinations."""
    n = len(keys)
    L = [(k >> bit) & 1 for k in keys]
    E = [1 - b for b in L]
    F = []
    acc = 0
    for e in E:
        F.append(acc)
        acc += e
    total_false = E[n - 1] + F[n - 1] if n else 0
    dest = [(i - F[i] + total_false) if L[i] else F[i] for i in range(n)]
    out = [None] * n
    for i, d in enumerate(dest):
        out[d] = keys[i]
    return {"L": L, "E": E, "F": F, "totalFalse": total_false, "dest": dest, "out": out}
