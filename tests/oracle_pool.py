"""The oracle over many independent pairs in parallel CPU worker processes
(test infrastructure: the workers import only numpy and the oracle, never
the GPU path). Pools use the spawn start method, so a worker never inherits
the parent's GPU runtime state."""
import multiprocessing as mp

import numpy as np


def pair_overlap(a: np.ndarray, b: np.ndarray) -> tuple:
    """The oracle's longest overlap of one pair (join, comparison-sort SA,
    direct LCP, overlap scan), on one thread."""
    import oracle
    offs = np.array([0, a.size, a.size + b.size], np.int64)
    joined = oracle.join(np.concatenate([a, b]) if a.size + b.size else np.zeros(0, np.uint8), offs)
    sa = oracle.suffix_array(joined, nthreads=1)
    return oracle.overlap(sa, oracle.lcp(joined, sa, nthreads=1), offs)


def pairs_overlap(pairs: list, procs: int = 16) -> list:
    with mp.get_context("spawn").Pool(procs) as pool:
        return pool.starmap(pair_overlap, pairs, chunksize=max(1, len(pairs) // (8 * procs)))
