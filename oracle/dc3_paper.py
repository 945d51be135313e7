"""The three DC3 steps of Section III, for tiny texts (test infrastructure only).

Used to pin the paper's worked example on `ATTGCTAC` (Tables I-III and the
step-2 ordering) and to check, on tiny inputs, that the steps reproduce the
suffix array defined by plain sorting. The text is a list of integers >= 1;
every position at or past the end reads as 0, which is smaller than every
symbol (the paper pads the last triple with zeros, e.g. "C00").

Readings of the paper encoded here (each is listed in the design notes):
  * the difference cover is taken over [0, v) and the non-sample class is B0;
  * R lists the mod-1 triples then the mod-2 triples, each in position order;
  * when n mod 3 == 1, a padding-only sample position n is added to the mod-1
    class, so the last mod-1 triple is unique and the suffixes of R that start
    in R1 stop before R2;
  * in the step-3 rule for B2 the ranks compared are those of S(i+2) and
    S(j+2) (the printed rule repeats i+1, which does not order the suffixes).
"""
from __future__ import annotations


def _at(t, i):
    return t[i] if i < len(t) else 0


def sample_positions(n: int) -> tuple:
    b1 = [i for i in range(1, n, 3)]
    if n % 3 == 1:
        b1.append(n)                     # padding-only sample position
    b2 = [i for i in range(2, n, 3)]
    return b1, b2


def name_triples(t, positions) -> list:
    """Lexicographic names (1-based) of the triples starting at positions."""
    trip = [(_at(t, i), _at(t, i + 1), _at(t, i + 2)) for i in positions]
    distinct = sorted(set(trip))
    name = {x: k + 1 for k, x in enumerate(distinct)}
    return [name[x] for x in trip]


def sample_ranks(t) -> dict:
    """Step 1: rank (1-based) of every sample suffix among the sample
    suffixes, including the padding-only position when present."""
    n = len(t)
    b1, b2 = sample_positions(n)
    pos = b1 + b2
    R = name_triples(t, pos)
    if len(set(R)) == len(R):
        rank_r = R
    else:
        sa_r = suffix_array(R)
        rank_r = [0] * len(R)
        for r, k in enumerate(sa_r):
            rank_r[k] = r + 1
    return {p: rank_r[k] for k, p in enumerate(pos)}


def real_sample_ranks(t) -> dict:
    """Ranks among the sample suffixes that start inside the text (Table II)."""
    ranks = sample_ranks(t)
    real = sorted((r, p) for p, r in ranks.items() if p < len(t))
    return {p: k + 1 for k, (r, p) in enumerate(real)}


def nonsample_order(t, ranks: dict) -> list:
    """Step 2: B0 ordered by the pair (t_i, rank(S_{i+1}))."""
    n = len(t)

    def rank(p):
        return ranks[p] if (p < n and p in ranks) else 0

    b0 = list(range(0, n, 3))
    return sorted(b0, key=lambda i: (_at(t, i), rank(i + 1)))


def suffix_array(t) -> list:
    """Steps 1-3 of DC3, recursing on R while triple names repeat."""
    n = len(t)
    if n == 0:
        return []
    if n == 1:
        return [0]
    ranks = sample_ranks(t)

    def rank(p):
        return ranks[p] if (p < n and p in ranks) else 0

    sample_sorted = sorted((p for p in ranks if p < n), key=lambda p: ranks[p])
    b0_sorted = nonsample_order(t, ranks)

    def sample_less(i, j):
        """Step 3: is sample suffix S_i smaller than non-sample suffix S_j?"""
        if i % 3 == 1:
            return (_at(t, i), rank(i + 1)) < (_at(t, j), rank(j + 1))
        return (_at(t, i), _at(t, i + 1), rank(i + 2)) < (_at(t, j), _at(t, j + 1), rank(j + 2))

    out = []
    a, b = 0, 0
    while a < len(sample_sorted) and b < len(b0_sorted):
        if sample_less(sample_sorted[a], b0_sorted[b]):
            out.append(sample_sorted[a])
            a += 1
        else:
            out.append(b0_sorted[b])
            b += 1
    out.extend(sample_sorted[a:])
    out.extend(b0_sorted[b:])
    return out
