"""The paper's radix-sort design (Section IV: one split per key bit inside
every chunk, then pairwise merges of the sorted chunks), through the C-ABI,
against numpy's stable argsort and the split example printed in Section IV."""
import sys

import numpy as np
import pytest

from paper_1404_3448_amd import ablation, lor

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def run_split(keys, vals, lo, hi):
    k = torch.from_numpy(np.ascontiguousarray(keys).view(np.int32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(vals)).cuda()
    lor.lor_sort_pairs_split_u32(k, v, lo, hi)
    torch.cuda.synchronize()
    return k.cpu().numpy().view(np.uint32), v.cpu().numpy()


def test_split_example_of_section_iv(golden):
    g = golden["paper_examples"]["split_example"]
    keys = np.array(g["keys"], np.uint32)
    vals = np.arange(keys.size, dtype=np.int32)
    k, v = run_split(keys, vals, g["bit"], g["bit"] + 1)
    assert k.tolist() == g["out"]
    dest = np.empty(keys.size, np.int64)
    dest[v] = np.arange(keys.size)        # where each input key went
    assert dest.tolist() == g["dest"]


# sizes around the chunk (2048), the wavefront (64) and the merge tiles;
# several merge passes and ragged tails
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 2047, 2048, 2049, 4096, 6143, 65536 + 64, 1_000_003, (1 << 22) + 7])
@pytest.mark.parametrize("bits", [(0, 32), (0, 1), (3, 17), (0, 15)])
def test_split_sort_matches_stable_argsort(n, bits):
    say("split sort", n, bits)
    rng = np.random.default_rng(n + 31 * bits[1])
    if bits == (0, 15):
        keys = rng.integers(0, 40, size=n).astype(np.uint32)          # heavy ties
    else:
        keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    vals = rng.permutation(n).astype(np.int32)
    lo, hi = bits
    digit = (keys.astype(np.uint64) >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1)
    order = np.argsort(digit, kind="stable")
    k, v = run_split(keys, vals, lo, hi)
    assert np.array_equal(k, keys[order])
    assert np.array_equal(v, vals[order])


def test_split_sort_on_level0_sample_keys_equals_digit_sort():
    keys = ablation.sample_keys(3 * 300_001)
    n = keys.size
    vals = np.arange(n, dtype=np.int32)
    k1, v1 = run_split(keys, vals, 0, 15)
    k = torch.from_numpy(keys.view(np.int32)).cuda()
    v = torch.from_numpy(vals).cuda()
    lor.lor_sort_pairs_u32(k, v, 0, 15)
    torch.cuda.synchronize()
    assert np.array_equal(k1, k.cpu().numpy().view(np.uint32))
    assert np.array_equal(v1, v.cpu().numpy())
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(v1, vals[order])
